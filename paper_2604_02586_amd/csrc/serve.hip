// tg_serve_*: the continuous-batching motion-transfer server (TrackerSplat
// Sec. 4.7, one GPU's share of the frame-parallel pipeline; the clip
// structure of Sec. 5.1).  Host C++ around the library's own entry points.
// Also tg_acc_zero, the accumulator fill both the server and a single frame
// use.
//
// Every target frame of a clip is transferred from the clip's first frame,
// so a stream (one clip) is projected and binned once when it is admitted and
// its splats and bins stay resident; its frames then only need their tracks,
// an accumulator array and one slot in a step.  A step is one
// tg_splat_accumulate_batch (alpha and T evaluated once per entry for all of
// its frames) and one tg_solve_triangulate_batch over every frame of the
// step, on the compute stream; track uploads run on the copy stream.
//
// Memory comes from one caller-owned device arena, sub-allocated here by a
// first-fit allocator over offsets (256-byte aligned, neighbours coalesced on
// release).  Admission is first in, first out: the head stream is admitted
// when its resident set (splats, bins, device cameras, binning workspace)
// and one frame's working set (accumulators, track copies) can all be
// allocated; that frame working set stays reserved for the stream's
// lifetime (its "credit"), so an admitted stream always progresses and the
// arena cannot deadlock.  Further frames allocate their own working sets as
// they fit; a block is released only after the event of the step (or
// binning) that last used it has completed.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "tg_internal.h"

namespace {

__global__ void __launch_bounds__(256) k_zero16(float4* __restrict__ p, int64_t n) {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = z;
}

// Zero n4 float4s: one store per thread over as many workgroups as it takes
// (a grid-stride loop over a capped grid writes HBM about 25% slower).
void launch_zero16(float4* p, int64_t n4, hipStream_t s) {
    if (n4 <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>((n4 + 255) / 256, INT64_C(1) << 30);
    hipLaunchKernelGGL(k_zero16, dim3(g), dim3(256), 0, s, p, n4);
}

constexpr uint64_t ALIGN = 256;
constexpr int READBACK_SLOTS = TG_SERVE_HOST_BYTES / 16;

uint64_t round_up(uint64_t b) { return (std::max<uint64_t>(b, 1) + ALIGN - 1) & ~(ALIGN - 1); }

// First-fit allocator over [0, size).
class Arena {
  public:
    explicit Arena(uint64_t size) : size_(size) {
        if (size_) free_[0] = size_;
    }
    int64_t alloc(uint64_t bytes) {
        bytes = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const uint64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return (int64_t)off;
        }
        return -1;
    }
    void release(int64_t off, uint64_t bytes) {
        if (off < 0) return;
        bytes = round_up(bytes);
        used_ -= bytes;
        auto it = free_.emplace((uint64_t)off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

  private:
    uint64_t size_;
    uint64_t used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Block {
    int64_t off = -1;
    uint64_t bytes = 0;
};

// Frame working set: accumulators and, for host tracks, their device copies.
struct WorkSet {
    Block acc, disp, vis;
};

enum class FState { Waiting, Ready, Running };
enum class CState { Waiting, Binning, Ready };

struct Frame {
    int64_t stream = 0, id = 0;
    const float* disp = nullptr;
    const uint8_t* vis = nullptr;
    bool host = false;
    tg_gaussians out{};
    uint32_t* status = nullptr;
    double arrival = 0.0;
    FState st = FState::Waiting;
    bool credit = false;       // runs on its stream's reserved working set
    WorkSet ws;                // own working set (credit == false)
    hipEvent_t up_ev = nullptr;
    int64_t step = -1;
    int entry = -1;
};

struct Clip {
    int64_t id = 0;
    tg_gaussians g{};
    int64_t N = 0;
    int V = 0, W = 0, H = 0;
    std::vector<tg_camera> cams;
    double opened = 0.0;
    bool admitted = false, closed = false;
    bool failed = false;         // its pair list can never fit the arena
    CState st = CState::Waiting;
    // resident set
    Block rec, cov2d, rect, key, order, cell_ids, cell_ranges, counters, cams_dev, ws;
    int64_t capacity = 0, n_cells = 0;
    uint64_t ws_bytes = 0;
    WorkSet credit;
    bool credit_free = true;
    hipEvent_t bin_ev = nullptr;
    int readback = -1;
    bool rebin_pending = false;
    std::deque<Frame*> frames;   // submitted and not yet done
    int64_t submitted = 0, finished = 0;
};

struct Entry {
    Clip* clip;
    std::vector<Frame*> frames;
};

struct Step {
    int64_t idx = 0;
    hipEvent_t ev = nullptr;
    std::vector<Entry> entries;
    bool dry_done = false;
    double dry_t = 0.0;
};

uint64_t frame_bytes_acc(const Clip& c) { return (uint64_t)c.V * (uint64_t)c.N * TG_ACC_STRIDE * 4; }
uint64_t frame_bytes_disp(const Clip& c) { return (uint64_t)c.V * c.H * c.W * 8; }
uint64_t frame_bytes_vis(const Clip& c) { return (uint64_t)c.V * c.H * c.W; }

// Resident set as allocated (splat records, covariances, rectangles, depth
// keys, depth order, pair list, bin ranges, counters, device cameras and the
// binning workspace), rounded as the arena rounds.
uint64_t resident_bytes(const Clip& c) {
    const uint64_t VN = (uint64_t)c.V * c.N;
    return round_up(VN * 32) + round_up(VN * 12) + round_up(VN * 8) + round_up(VN * 4) + round_up(VN * 4) +
           round_up((uint64_t)std::max<int64_t>(c.capacity, 1) * 4) + round_up((uint64_t)c.n_cells * 8) +
           round_up(16) + round_up((uint64_t)c.V * sizeof(tg_camera)) + round_up(c.ws_bytes);
}

// One frame's working set: accumulators, and track copies for host tracks.
uint64_t frame_set_bytes(const Clip& c, bool host) {
    return round_up(frame_bytes_acc(c)) + (host ? round_up(frame_bytes_disp(c)) + round_up(frame_bytes_vis(c)) : 0);
}

// Sizes a stream from its description alone (no device), as the server
// does when the stream is opened.
tg_status describe(Clip& c, const tg_gaussians* g, int64_t N, const tg_camera* cams, int V, const tg_params* prm) {
    if (V < 1 || N < 0) return TG_ERR_INVALID_ARG;
    if (V > TG_MAX_VIEWS || N > (int64_t)0xFFFFFFFF) return TG_ERR_UNSUPPORTED;
    for (int v = 1; v < V; ++v)
        if (cams[v].width != cams[0].width || cams[v].height != cams[0].height) return TG_ERR_INVALID_ARG;
    if (cams[0].width < 1 || cams[0].height < 1) return TG_ERR_INVALID_ARG;
    if (g) {
        c.g = *g;
        c.g.sh = nullptr;
    }
    c.N = N;
    c.V = V;
    c.W = cams[0].width;
    c.H = cams[0].height;
    c.cams.assign(cams, cams + V);
    c.n_cells = tg_num_cells(cams, V, std::max<int64_t>(N, 1), prm);
    if (c.n_cells < 0) return TG_ERR_UNSUPPORTED;
    // first guess of the pair count: a few coarse bins per (view, Gaussian);
    // an overflow re-bins with the exact count
    c.capacity = std::max<int64_t>(1024, 3 * N * V);
    tg_splats s{};
    tg_bins b{};
    b.capacity = c.capacity;
    size_t wsb = 0;
    const tg_status st = tg_bin_sort(&s, std::max<int64_t>(N, 1), cams, V, prm, &b, nullptr, &wsb, nullptr);
    if (st != TG_OK) return st;
    c.ws_bytes = wsb;
    return TG_OK;
}

}  // namespace

struct tg_server {
    tg_serve_config cfg{};
    tg_params prm{};
    Arena arena{0};
    char* base = nullptr;
    hipStream_t comp = nullptr, copy = nullptr;
    bool dry = false;
    std::map<int64_t, Clip*> clips;
    std::deque<Clip*> queue;            // opened, not yet admitted (FIFO)
    std::deque<Step*> inflight;
    std::deque<tg_serve_done> done;
    std::vector<hipEvent_t> sync_pool, timing_pool;
    bool readback_used[READBACK_SLOTS] = {};
    hipEvent_t t0_ev = nullptr;
    std::chrono::steady_clock::time_point t0;
    int64_t next_id = 0, next_step = 0;
    tg_serve_stats stats{};

    ~tg_server() {
        for (auto& kv : clips) {
            for (Frame* f : kv.second->frames) delete f;
            delete kv.second;
        }
        for (Step* s : inflight) delete s;
        if (!dry) {
            for (hipEvent_t e : sync_pool) (void)hipEventDestroy(e);
            for (hipEvent_t e : timing_pool) (void)hipEventDestroy(e);
            if (t0_ev) (void)hipEventDestroy(t0_ev);
        }
    }

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void* ptr(const Block& b) const { return b.off < 0 ? nullptr : (void*)(base + b.off); }

    // ---- events (reused)
    tg_status get_event(bool timing, hipEvent_t* e) {
        *e = nullptr;
        if (dry) return TG_OK;
        auto& pool = timing ? timing_pool : sync_pool;
        if (!pool.empty()) {
            *e = pool.back();
            pool.pop_back();
            return TG_OK;
        }
        const unsigned flags = timing ? hipEventDefault : hipEventDisableTiming;
        return hipEventCreateWithFlags(e, flags) == hipSuccess ? TG_OK : TG_ERR_DEVICE;
    }
    void put_event(bool timing, hipEvent_t e) {
        if (e) (timing ? timing_pool : sync_pool).push_back(e);
    }
    // 1: complete, 0: not yet, -1: error
    int query(hipEvent_t e) const {
        if (dry || !e) return 1;
        const hipError_t r = hipEventQuery(e);
        if (r == hipSuccess) return 1;
        if (r == hipErrorNotReady) return 0;
        return -1;
    }

    // ---- all-or-nothing allocation of a list of blocks
    bool alloc_all(std::initializer_list<std::pair<Block*, uint64_t>> req) {
        std::vector<Block*> got;
        for (auto& r : req) {
            if (r.second == 0) {
                *r.first = Block{};
                continue;
            }
            const int64_t off = arena.alloc(r.second);
            if (off < 0) {
                for (Block* b : got) free_block(*b);
                return false;
            }
            *r.first = Block{off, r.second};
            got.push_back(r.first);
        }
        return true;
    }
    void free_block(Block& b) {
        if (b.off >= 0) arena.release(b.off, b.bytes);
        b = Block{};
    }
    void free_workset(WorkSet& w) {
        free_block(w.acc);
        free_block(w.disp);
        free_block(w.vis);
    }
    bool alloc_workset(const Clip& c, WorkSet& w, bool host) {
        return alloc_all({{&w.acc, frame_bytes_acc(c)},
                          {&w.disp, host ? frame_bytes_disp(c) : 0},
                          {&w.vis, host ? frame_bytes_vis(c) : 0}});
    }

    uint64_t admit_bytes(const Clip& c) const { return resident_bytes(c) + frame_set_bytes(c, true); }

    tg_splats splats(const Clip& c) const {
        tg_splats s{};
        s.rec = (float*)ptr(c.rec);
        s.cov2d = (float*)ptr(c.cov2d);
        s.rect = (uint16_t*)ptr(c.rect);
        s.key = (uint32_t*)ptr(c.key);
        return s;
    }
    tg_bins bins(const Clip& c) const {
        tg_bins b{};
        b.order = (uint32_t*)ptr(c.order);
        b.cell_ids = (uint32_t*)ptr(c.cell_ids);
        b.cell_ranges = (uint32_t*)ptr(c.cell_ranges);
        b.n_pairs = (int64_t*)ptr(c.counters);
        b.overflow = (int32_t*)((char*)ptr(c.counters) + 8);
        b.capacity = c.capacity;
        return b;
    }

    // ---- binning of an admitted stream (projection included); the pair
    // count and overflow flag come back through a pinned read-back slot
    tg_status launch_binning(Clip& c) {
        if (dry) {
            c.st = CState::Ready;
            free_block(c.ws);
            return TG_OK;
        }
        tg_splats s = splats(c);
        tg_bins b = bins(c);
        tg_status st = tg_preprocess(&c.g, c.N, c.cams.data(), c.V, &prm, &s, comp);
        if (st != TG_OK) return st;
        size_t wsb = c.ws_bytes;
        st = tg_bin_sort(&s, c.N, c.cams.data(), c.V, &prm, &b, ptr(c.ws), &wsb, comp);
        if (st != TG_OK) return st;
        char* slot = (char*)cfg.host_scratch + 16 * c.readback;
        if (hipMemcpyAsync(slot, b.n_pairs, 8, hipMemcpyDeviceToHost, comp) != hipSuccess ||
            hipMemcpyAsync(slot + 8, b.overflow, 4, hipMemcpyDeviceToHost, comp) != hipSuccess)
            return TG_ERR_DEVICE;
        if (!c.bin_ev && get_event(false, &c.bin_ev) != TG_OK) return TG_ERR_DEVICE;
        if (hipEventRecord(c.bin_ev, comp) != hipSuccess) return TG_ERR_DEVICE;
        c.st = CState::Binning;
        return TG_OK;
    }

    int take_readback() {
        for (int i = 0; i < READBACK_SLOTS; ++i)
            if (!readback_used[i]) {
                readback_used[i] = true;
                return i;
            }
        return -1;
    }

    // ---- steps ------------------------------------------------------------
    tg_status retire() {
        while (!inflight.empty()) {
            Step* s = inflight.front();
            double t;
            if (dry) {
                if (!s->dry_done) break;
                t = s->dry_t;
            } else {
                const int q = query(s->ev);
                if (q < 0) return TG_ERR_DEVICE;
                if (q == 0) break;
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, t0_ev, s->ev) != hipSuccess) return TG_ERR_DEVICE;
                t = ms * 1e-3;
            }
            inflight.pop_front();
            for (Entry& e : s->entries) {
                Clip* c = e.clip;
                for (Frame* f : e.frames) {
                    done.push_back(tg_serve_done{f->stream, f->id, f->step, f->arrival, t, TG_OK, f->entry});
                    if (f->credit)
                        c->credit_free = true;
                    else
                        free_workset(f->ws);
                    put_event(false, f->up_ev);
                    c->frames.erase(std::find(c->frames.begin(), c->frames.end(), f));
                    delete f;
                    ++c->finished;
                }
            }
            put_event(true, s->ev);
            delete s;
        }
        return sweep();
    }

    // Streams that failed report their frames (once no upload into their
    // working sets is in flight); closed streams whose last frame is done
    // and whose binning has finished release their resident sets.
    tg_status sweep() {
        for (auto it = clips.begin(); it != clips.end();) {
            Clip* c = it->second;
            if (c->failed) {
                for (auto fi = c->frames.begin(); fi != c->frames.end();) {
                    Frame* f = *fi;
                    const int q = query(f->up_ev);
                    if (q < 0) return TG_ERR_DEVICE;
                    if (q == 0) {
                        ++fi;
                        continue;
                    }
                    done.push_back(tg_serve_done{f->stream, f->id, -1, f->arrival, now(), TG_ERR_BUDGET, -1});
                    if (f->credit)
                        c->credit_free = true;
                    else
                        free_workset(f->ws);
                    put_event(false, f->up_ev);
                    delete f;
                    fi = c->frames.erase(fi);
                    ++c->finished;
                }
            }
            if (c->admitted && c->closed && c->frames.empty() && (c->st == CState::Ready || c->failed)) {
                release_clip(*c);
                delete c;
                it = clips.erase(it);
            } else {
                ++it;
            }
        }
        return TG_OK;
    }

    void release_clip(Clip& c) {
        for (Block* b : {&c.rec, &c.cov2d, &c.rect, &c.key, &c.order, &c.cell_ids, &c.cell_ranges, &c.counters,
                         &c.cams_dev, &c.ws})
            free_block(*b);
        free_workset(c.credit);
        put_event(false, c.bin_ev);
        c.bin_ev = nullptr;
        if (c.readback >= 0) readback_used[c.readback] = false;
        c.readback = -1;
    }

    tg_status check_bins() {
        for (auto& kv : clips) {
            Clip& c = *kv.second;
            if (!c.admitted || c.st != CState::Binning || c.failed) continue;
            if (c.rebin_pending) {
                // a larger pair list and its workspace, allocated as they fit
                if (!alloc_all({{&c.cell_ids, (uint64_t)c.capacity * 4}, {&c.ws, c.ws_bytes}})) continue;
                c.rebin_pending = false;
                tg_status st = launch_binning(c);
                if (st != TG_OK) return st;
                continue;
            }
            const int q = query(c.bin_ev);
            if (q < 0) return TG_ERR_DEVICE;
            if (q == 0) continue;
            const char* slot = (const char*)cfg.host_scratch + 16 * c.readback;
            int64_t n_pairs;
            int32_t overflow;
            memcpy(&n_pairs, slot, 8);
            memcpy(&overflow, slot + 8, 4);
            if (overflow) {
                ++stats.rebins;
                free_block(c.cell_ids);
                free_block(c.ws);
                c.capacity = n_pairs + n_pairs / 10 + 1024;
                size_t wsb = 0;
                tg_splats s = splats(c);
                tg_bins b = bins(c);
                b.capacity = c.capacity;
                if (tg_bin_sort(&s, c.N, c.cams.data(), c.V, &prm, &b, nullptr, &wsb, comp) != TG_OK)
                    return TG_ERR_UNSUPPORTED;
                c.ws_bytes = wsb;
                if (admit_bytes(c) > arena.size()) {
                    c.failed = true;   // its frames end with TG_ERR_BUDGET
                    readback_used[c.readback] = false;
                    c.readback = -1;
                    continue;
                }
                c.rebin_pending = true;
                continue;
            }
            c.st = CState::Ready;
            free_block(c.ws);   // the workspace is only needed while binning
            readback_used[c.readback] = false;
            c.readback = -1;
        }
        return TG_OK;
    }

    tg_status admit() {
        while (!queue.empty()) {
            Clip& c = *queue.front();
            const int rb = dry ? 0 : take_readback();
            if (rb < 0) break;
            const uint64_t VN = (uint64_t)c.V * c.N;
            const bool ok = alloc_all({{&c.rec, VN * 32},
                                       {&c.cov2d, VN * 12},
                                       {&c.rect, VN * 8},
                                       {&c.key, VN * 4},
                                       {&c.order, VN * 4},
                                       {&c.cell_ids, (uint64_t)std::max<int64_t>(c.capacity, 1) * 4},
                                       {&c.cell_ranges, (uint64_t)c.n_cells * 8},
                                       {&c.counters, 16},
                                       {&c.cams_dev, (uint64_t)c.V * sizeof(tg_camera)},
                                       {&c.ws, c.ws_bytes}});
            if (!ok) {
                if (!dry) readback_used[rb] = false;
                break;
            }
            if (!alloc_workset(c, c.credit, true)) {
                release_clip(c);
                if (!dry) readback_used[rb] = false;
                break;
            }
            c.readback = dry ? -1 : rb;
            queue.pop_front();
            c.admitted = true;
            if (!dry && hipMemcpyAsync(ptr(c.cams_dev), c.cams.data(), (size_t)c.V * sizeof(tg_camera),
                                       hipMemcpyHostToDevice, comp) != hipSuccess)
                return TG_ERR_DEVICE;
            tg_status st = launch_binning(c);
            if (st != TG_OK) return st;
        }
        int64_t adm = 0;
        for (auto& kv : clips) adm += kv.second->admitted ? 1 : 0;
        stats.max_admitted = std::max(stats.max_admitted, adm);
        return TG_OK;
    }

    tg_status upload() {
        std::vector<Frame*> fr;
        for (auto& kv : clips)
            if (kv.second->admitted && !kv.second->failed)
                for (Frame* f : kv.second->frames)
                    if (f->st == FState::Waiting) fr.push_back(f);
        std::stable_sort(fr.begin(), fr.end(), [](const Frame* a, const Frame* b) { return a->arrival < b->arrival; });
        for (Frame* f : fr) {
            Clip& c = *clips[f->stream];
            if (c.credit_free) {
                c.credit_free = false;
                f->credit = true;
            } else if (!alloc_workset(c, f->ws, f->host)) {
                break;   // oldest first: no overtaking of a frame that does not fit
            }
            if (f->host && !dry) {
                const WorkSet& w = f->credit ? c.credit : f->ws;
                if (hipMemcpyAsync(ptr(w.disp), f->disp, frame_bytes_disp(c), hipMemcpyHostToDevice, copy) !=
                    hipSuccess)
                    return TG_ERR_DEVICE;
                if (f->vis && hipMemcpyAsync(ptr(w.vis), f->vis, frame_bytes_vis(c), hipMemcpyHostToDevice, copy) !=
                                  hipSuccess)
                    return TG_ERR_DEVICE;
                if (get_event(false, &f->up_ev) != TG_OK || hipEventRecord(f->up_ev, copy) != hipSuccess)
                    return TG_ERR_DEVICE;
            }
            f->st = FState::Ready;
        }
        return TG_OK;
    }

    const WorkSet& workset(const Clip& c, const Frame& f) const { return f.credit ? c.credit : f.ws; }

    // The streams whose oldest ready frame is oldest; up to max_frames of a
    // stream's ready frames in entries of at most TG_MAX_FRAMES; up to
    // max_slots entries.
    std::vector<Entry> compose() {
        struct Cand {
            double t;
            int64_t id;
            Clip* c;
            std::vector<Frame*> fr;
        };
        std::vector<Cand> cands;
        for (auto& kv : clips) {
            Clip* c = kv.second;
            if (!c->admitted || c->st != CState::Ready) continue;
            std::vector<Frame*> fr;
            for (Frame* f : c->frames)
                if (f->st == FState::Ready) fr.push_back(f);
            if (fr.empty()) continue;
            std::stable_sort(fr.begin(), fr.end(),
                             [](const Frame* a, const Frame* b) { return a->arrival < b->arrival; });
            if ((int)fr.size() > cfg.max_frames) fr.resize(cfg.max_frames);
            cands.push_back(Cand{fr[0]->arrival, c->id, c, fr});
        }
        std::sort(cands.begin(), cands.end(),
                  [](const Cand& a, const Cand& b) { return a.t < b.t || (a.t == b.t && a.id < b.id); });
        std::vector<Entry> out;
        for (Cand& cd : cands) {
            for (size_t i = 0; i < cd.fr.size() && (int)out.size() < cfg.max_slots; i += TG_MAX_FRAMES) {
                Entry e{cd.c, {}};
                for (size_t j = i; j < std::min(cd.fr.size(), i + TG_MAX_FRAMES); ++j) e.frames.push_back(cd.fr[j]);
                out.push_back(std::move(e));
            }
            if ((int)out.size() >= cfg.max_slots) break;
        }
        return out;
    }

    tg_status launch_step(std::vector<Entry>& entries) {
        Step* s = new (std::nothrow) Step();
        if (!s) return TG_ERR_DEVICE;
        s->idx = next_step++;
        int64_t nfr = 0;
        for (size_t k = 0; k < entries.size(); ++k)
            for (Frame* f : entries[k].frames) {
                f->st = FState::Running;
                f->step = s->idx;
                f->entry = (int)k;
                ++nfr;
            }
        s->entries = std::move(entries);
        if (!dry) {
            std::vector<tg_acc_slot> acc(s->entries.size());
            std::vector<tg_upd_slot> upd(s->entries.size());
            std::vector<tg_splats> sp(s->entries.size());
            std::vector<tg_bins> bn(s->entries.size());
            for (size_t k = 0; k < s->entries.size(); ++k) {
                Entry& e = s->entries[k];
                Clip& c = *e.clip;
                sp[k] = splats(c);
                bn[k] = bins(c);
                acc[k] = tg_acc_slot{};
                acc[k].s = &sp[k];
                acc[k].bins = &bn[k];
                acc[k].cams = c.cams.data();
                acc[k].N = c.N;
                acc[k].V = c.V;
                acc[k].F = (int32_t)e.frames.size();
                upd[k] = tg_upd_slot{};
                upd[k].s = &sp[k];
                upd[k].g_in = &c.g;
                upd[k].cams = (const tg_camera*)ptr(c.cams_dev);
                upd[k].N = c.N;
                upd[k].V = c.V;
                upd[k].F = (int32_t)e.frames.size();
                for (size_t j = 0; j < e.frames.size(); ++j) {
                    Frame& f = *e.frames[j];
                    const WorkSet& w = workset(c, f);
                    float* a = (float*)ptr(w.acc);
                    launch_zero16((float4*)a, (int64_t)(frame_bytes_acc(c) / 16), comp);
                    if (f.up_ev && hipStreamWaitEvent(comp, f.up_ev, 0) != hipSuccess) return TG_ERR_DEVICE;
                    acc[k].disp[j] = f.host ? (const float*)ptr(w.disp) : f.disp;
                    acc[k].vis[j] = f.vis ? (f.host ? (const uint8_t*)ptr(w.vis) : f.vis) : nullptr;
                    acc[k].acc[j] = a;
                    upd[k].acc[j] = a;
                    upd[k].g_out[j] = &f.out;
                    upd[k].status[j] = f.status;
                }
            }
            TG_CHECK_LAUNCH();
            tg_status st = tg_splat_accumulate_batch(acc.data(), (int32_t)acc.size(), &prm, nullptr, comp);
            if (st != TG_OK) return st;
            st = tg_solve_triangulate_batch(upd.data(), (int32_t)upd.size(), &prm, comp);
            if (st != TG_OK) return st;
            if (get_event(true, &s->ev) != TG_OK || hipEventRecord(s->ev, comp) != hipSuccess) return TG_ERR_DEVICE;
        }
        inflight.push_back(s);
        ++stats.steps;
        stats.entries += (int64_t)s->entries.size();
        stats.frames += nfr;
        return TG_OK;
    }
};

// ---------------------------------------------------------------- C ABI
extern "C" tg_status tg_acc_zero(float* acc, int64_t n_records, void* stream)
{
    if (n_records < 0 || n_records > INT64_MAX / 64 || (n_records > 0 && !acc)) return TG_ERR_INVALID_ARG;
    if (n_records == 0) return TG_OK;
    if (!aligned16(acc)) return TG_ERR_ALIGNMENT;
    launch_zero16((float4*)acc, n_records * (TG_ACC_STRIDE / 4), (hipStream_t)stream);
    TG_CHECK_LAUNCH();
    return TG_OK;
}

extern "C" tg_status tg_serve_create(const tg_serve_config* cfg, const tg_params* p, tg_server** out) {
    if (!cfg || !p || !out) return TG_ERR_INVALID_ARG;
    *out = nullptr;
    const bool dry = cfg->dry != 0;
    if (cfg->max_inflight < 1 || cfg->max_frames < 1 || cfg->max_frames > 2 * TG_MAX_FRAMES ||
        cfg->max_slots < 1 || cfg->max_slots > TG_MAX_SLOTS)
        return TG_ERR_INVALID_ARG;
    if (dry ? cfg->arena != nullptr : (!cfg->arena || !cfg->host_scratch)) return TG_ERR_INVALID_ARG;
    if (((uintptr_t)cfg->arena & (ALIGN - 1)) != 0) return TG_ERR_ALIGNMENT;
    tg_server* s = new (std::nothrow) tg_server();
    if (!s) return TG_ERR_DEVICE;
    s->cfg = *cfg;
    s->prm = *p;
    s->dry = dry;
    s->arena = Arena(cfg->arena_bytes & ~(ALIGN - 1));
    s->base = dry ? (char*)nullptr : (char*)cfg->arena;
    s->comp = (hipStream_t)cfg->compute_stream;
    s->copy = cfg->copy_stream ? (hipStream_t)cfg->copy_stream : s->comp;
    if (!dry) {
        // a common origin for host and GPU times: the GPU reaches t0_ev just
        // before the host reads its clock
        if (hipEventCreateWithFlags(&s->t0_ev, hipEventDefault) != hipSuccess ||
            hipEventRecord(s->t0_ev, s->comp) != hipSuccess || hipEventSynchronize(s->t0_ev) != hipSuccess) {
            delete s;
            return TG_ERR_DEVICE;
        }
    }
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return TG_OK;
}

extern "C" tg_status tg_serve_destroy(tg_server* srv) {
    if (!srv) return TG_ERR_INVALID_ARG;
    tg_status st = TG_OK;
    if (!srv->dry) {
        for (Step* s : srv->inflight)
            if (s->ev && hipEventSynchronize(s->ev) != hipSuccess) st = TG_ERR_DEVICE;
        for (auto& kv : srv->clips)
            if (kv.second->bin_ev && hipEventSynchronize(kv.second->bin_ev) != hipSuccess) st = TG_ERR_DEVICE;
        if (hipStreamSynchronize(srv->copy) != hipSuccess) st = TG_ERR_DEVICE;
    }
    delete srv;
    return st;
}

extern "C" double tg_serve_now(const tg_server* srv) { return srv ? srv->now() : 0.0; }

extern "C" tg_status tg_serve_open_stream(tg_server* srv, const tg_gaussians* g, int64_t N, const tg_camera* cams,
                                          int32_t V, double arrival, int64_t* stream_id) {
    if (!srv || !g || !cams || !stream_id) return TG_ERR_INVALID_ARG;
    if (!srv->dry && (!g->means || !g->quats || !g->scales || !g->opacity)) return TG_ERR_INVALID_ARG;
    if (g->scale_mode < 0 || g->scale_mode > 1 || g->opacity_mode < 0 || g->opacity_mode > 1)
        return TG_ERR_INVALID_ARG;
    Clip* c = new (std::nothrow) Clip();
    if (!c) return TG_ERR_DEVICE;
    const tg_status st = describe(*c, g, N, cams, V, &srv->prm);
    if (st != TG_OK) {
        delete c;
        return st;
    }
    c->id = srv->next_id++;
    c->opened = arrival;
    if (srv->admit_bytes(*c) > srv->arena.size()) {
        delete c;
        return TG_ERR_BUDGET;
    }
    srv->clips[c->id] = c;
    srv->queue.push_back(c);
    *stream_id = c->id;
    return TG_OK;
}

extern "C" tg_status tg_serve_submit(tg_server* srv, int64_t stream_id, int64_t frame_id, const float* disp,
                                     const uint8_t* vis, int32_t host_tracks, tg_gaussians* g_out, uint32_t* status,
                                     double arrival) {
    if (!srv || !g_out) return TG_ERR_INVALID_ARG;
    auto it = srv->clips.find(stream_id);
    if (it == srv->clips.end() || it->second->closed) return TG_ERR_INVALID_ARG;
    if (!srv->dry && (!disp || !g_out->means || !g_out->quats || !g_out->scales)) return TG_ERR_INVALID_ARG;
    Frame* f = new (std::nothrow) Frame();
    if (!f) return TG_ERR_DEVICE;
    f->stream = stream_id;
    f->id = frame_id;
    f->disp = disp;
    f->vis = vis;
    f->host = host_tracks != 0;
    f->out = *g_out;
    f->status = status;
    f->arrival = arrival;
    it->second->frames.push_back(f);
    ++it->second->submitted;
    return TG_OK;
}

extern "C" tg_status tg_serve_close_stream(tg_server* srv, int64_t stream_id) {
    if (!srv) return TG_ERR_INVALID_ARG;
    auto it = srv->clips.find(stream_id);
    if (it == srv->clips.end() || it->second->closed) return TG_ERR_INVALID_ARG;
    Clip* c = it->second;
    c->closed = true;
    if (!c->admitted && c->frames.empty()) {
        // never admitted and nothing to do: withdrawn from the queue
        srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), c));
        delete c;
        srv->clips.erase(it);
        return TG_OK;
    }
    return srv->sweep();
}

extern "C" tg_status tg_serve_step(tg_server* srv, int32_t* launched) {
    if (!srv) return TG_ERR_INVALID_ARG;
    if (launched) *launched = 0;
    tg_status st;
    if ((st = srv->retire()) != TG_OK) return st;
    if ((st = srv->check_bins()) != TG_OK) return st;
    if ((st = srv->admit()) != TG_OK) return st;
    if ((st = srv->upload()) != TG_OK) return st;
    int32_t n = 0;
    while ((int)srv->inflight.size() < srv->cfg.max_inflight) {
        std::vector<Entry> e = srv->compose();
        if (e.empty()) break;
        if ((st = srv->launch_step(e)) != TG_OK) return st;
        ++n;
    }
    if (launched) *launched = n;
    return TG_OK;
}

extern "C" tg_status tg_serve_poll(tg_server* srv, tg_serve_done* out, int32_t max, int32_t* n) {
    if (!srv || !n || max < 0 || (max > 0 && !out)) return TG_ERR_INVALID_ARG;
    tg_status st = srv->retire();
    int32_t k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    *n = k;
    return st;
}

extern "C" tg_status tg_serve_get_stats(const tg_server* srv, tg_serve_stats* st) {
    if (!srv || !st) return TG_ERR_INVALID_ARG;
    *st = srv->stats;
    st->arena_used = (int64_t)srv->arena.used();
    st->arena_peak = (int64_t)srv->arena.peak();
    st->waiting_streams = (int64_t)srv->queue.size();
    int64_t adm = 0;
    for (auto& kv : srv->clips) adm += kv.second->admitted ? 1 : 0;
    st->admitted_streams = adm;
    st->inflight_steps = (int64_t)srv->inflight.size();
    return TG_OK;
}

extern "C" tg_status tg_serve_dry_complete(tg_server* srv, int32_t n, double now) {
    if (!srv || !srv->dry || n < 0) return TG_ERR_INVALID_ARG;
    for (Step* s : srv->inflight) {
        if (n == 0) break;
        if (s->dry_done) continue;
        s->dry_done = true;
        s->dry_t = now;
        --n;
    }
    return TG_OK;
}

extern "C" tg_status tg_serve_stream_bytes(const tg_camera* cams, int32_t V, int64_t N, const tg_params* p,
                                           int64_t* resident, int64_t* frame_host, int64_t* frame_device) {
    if (!cams || !p) return TG_ERR_INVALID_ARG;
    Clip c;
    const tg_status st = describe(c, nullptr, N, cams, V, p);
    if (st != TG_OK) return st;
    if (resident) *resident = (int64_t)resident_bytes(c);
    if (frame_host) *frame_host = (int64_t)frame_set_bytes(c, true);
    if (frame_device) *frame_device = (int64_t)frame_set_bytes(c, false);
    return TG_OK;
}
