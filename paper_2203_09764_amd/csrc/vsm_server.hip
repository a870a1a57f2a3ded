// vsm_server.hip -- the serving scheduler of include/vsm.h: a FIFO of smoothing
// jobs admitted by memory footprint into resident slots, and a worker thread
// that drives two streams.  Lattices above kSmallSites advance by one annealing
// subset pass per step, all such jobs of a step in one batched launch; small
// lattices advance by whole sweeps per step, each job inside one workgroup of a
// persistent launch (k_serve_small) on a second stream, so that their many
// short passes neither cost a launch each nor wait for the large jobs' steps.
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vsm.h"
#include "vsm_host.h"
#include "vsm_launch.h"

using namespace vsm;

namespace {

// First-fit allocator of offsets in a fixed region; free ranges are merged
// with their neighbours on release.  Not thread-safe (the server's mutex
// guards it).
class Arena {
 public:
  explicit Arena(size_t cap) : cap_(cap) {
    if (cap_) free_[0] = cap_;
  }
  bool alloc(size_t n, size_t* off) {
    n = align256(n ? n : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n;
      const size_t at = it->first + n;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += n;
      if (used_ > peak_) peak_ = used_;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align256(n ? n : 1);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
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
  size_t peak() const { return peak_; }

 private:
  size_t cap_, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
};

// Byte layout of one job in the device pool and in the pinned host pool.
struct JobLayout {
  size_t links, z3, pairs, ws, records, canon, dev_total;  // device offsets
  size_t h_in_z3, h_in_pairs, h_records, h_links, host_total;  // host offsets
};

int n_records_of(const vsm_job& j) {
  if (j.measure_every <= 0) return 1;
  return j.n_sweeps / j.measure_every + (j.n_sweeps % j.measure_every ? 1 : 0);
}

JobLayout layout_of(const vsm_job& j) {
  const Geo g = make_geo(j.dims);
  const size_t V = g.V;
  JobLayout L;
  size_t o = 0;
  L.links = o;
  o += align256(24ull * g.es * entry_bytes(j.precision));
  L.z3 = o;
  o += align256(4ull * V);
  L.pairs = o;
  if (j.pair_host) o += align256(4ull * V);
  L.ws = o;
  o += align256(ws_layout(j.dims, j.precision, VSM_ANNEALED).total);
  L.records = o;
  o += align256((size_t)n_records_of(j) * sizeof(vsm_stats));
  L.canon = o;
  if (j.want_links) o += align256(4ull * V * 9 * 16);
  L.dev_total = o;
  size_t h = 0;
  L.h_in_z3 = h;
  h += align256(4ull * V);
  L.h_in_pairs = h;
  if (j.pair_host) h += align256(4ull * V);
  L.h_records = h;
  h += align256((size_t)n_records_of(j) * sizeof(vsm_stats));
  L.h_links = h;
  if (j.want_links) h += align256(4ull * V * 9 * 16);
  L.host_total = h;
  return L;
}

int validate_job(const vsm_job* j) {
  if (!j || !j->z3_host) return VSM_E_NULL;
  int rc = check_sched(&j->sched);
  if (rc) return rc;
  if (j->sched.order != VSM_ANNEALED || j->sched.update != VSM_STOUT) return VSM_E_PARAM;
  rc = check_dims_impl(j->dims, VSM_ANNEALED, j->precision);
  if (rc) return rc;
  if (j->n_sweeps < 0 || j->measure_every < 0 || !is_fin(j->rho) || !is_fin(j->eps)) return VSM_E_PARAM;
  if (j->n_sweeps > (1 << 26)) return VSM_E_PARAM;
  if (j->pair_host && (!is_fin(j->omega) || !(fabs(j->omega) < 0.25))) return VSM_E_PARAM;
  return VSM_OK;
}

struct Job {
  uint64_t id = 0;
  vsm_job desc{};
  std::vector<int8_t> z3, pairs;  // host copies until the job is admitted
  Geo g{};
  UpdParams p{};
  JobLayout lay{};
  size_t dev_off = 0, host_off = 0;
  bool has_dev = false, has_host = false;
  int slot = -1;
  int state = VSM_JOB_QUEUED, status = VSM_OK;
  int n_records = 0, rec = 0;
  int64_t pass = 0, n_pass = 0;
  bool small = false;      // served by the small-lattice path
  hipStream_t st = nullptr;  // the stream all of the job's device work goes to
  double t_submit = -1, t_admit = -1, t_done = -1;
  hipEvent_t done_ev = nullptr;
  char* dbase = nullptr;
  char* hbase = nullptr;
};

class Server {
 public:
  vsm_server_config cfg{};
  hipStream_t stream = nullptr;        // large lattices: batched pass steps
  hipStream_t stream_small = nullptr;  // small lattices: whole-sweep workgroup steps
  char* dev_pool = nullptr;
  char* host_pool = nullptr;
  ServeJob* jobs_dev = nullptr;
  ServeJob* desc_host = nullptr;  // pinned staging of the job descriptors, one per slot
  std::vector<hipEvent_t> step_ev, small_ev;
  std::unique_ptr<Arena> dev_arena, host_arena;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
  std::deque<Job*> queue, running, running_small, finishing;
  std::vector<int> free_slots;
  uint64_t next_id = 1;
  uint64_t gen = 0;  // bumped by submit and fetch: the queue head may now fit
  bool stopping = false;
  int broken = VSM_OK;
  vsm_server_counters ctr{};
  std::chrono::steady_clock::time_point t0;
  std::thread worker;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // ---- worker side (called with mu held unless stated)

  void fail_job(Job* j, int status) {
    j->state = VSM_JOB_FAILED;
    j->status = status;
    j->t_done = now();
    ++ctr.jobs_failed;
  }

  // Frees the device side of a job whose device work has completed.
  void release_device(Job* j) {
    if (j->has_dev) dev_arena->release(j->dev_off, j->lay.dev_total);
    j->has_dev = false;
    if (j->slot >= 0) free_slots.push_back(j->slot);
    j->slot = -1;
    if (j->done_ev) (void)hipEventDestroy(j->done_ev);
    j->done_ev = nullptr;
  }

  int enqueue_measure(Job* j, long long sweep) {
    char* d = j->dbase;
    const WsLayout w = ws_layout(j->desc.dims, j->desc.precision, VSM_ANNEALED);
    launch_measure(j->desc.precision, j->g, d + j->lay.links, (const int8_t*)(d + j->lay.ws + w.charges),
                   nullptr, d + j->lay.ws + w.partials, nullptr, (unsigned long long*)(d + j->lay.ws),
                   (VsmStatsDev*)(d + j->lay.records) + j->rec, sweep, j->st);
    ++j->rec;
    ++ctr.launches;
    return hip_status();
  }

  // Final record, final links and the copies of the results to the pinned host
  // pool, then the job's completion event.
  int enqueue_finish(Job* j) {
    int rc = VSM_OK;
    if (j->rec < j->n_records) rc = enqueue_measure(j, j->desc.n_sweeps);
    char* d = j->dbase;
    if (!rc && j->desc.want_links) {
      launch_get_links(j->desc.precision, j->g, d + j->lay.links, d + j->lay.canon, j->st);
      ++ctr.launches;
      rc = hip_status();
    }
    hipError_t e = hipSuccess;
    if (!rc && j->n_records > 0)
      e = hipMemcpyAsync(j->hbase + j->lay.h_records, d + j->lay.records,
                         (size_t)j->n_records * sizeof(vsm_stats), hipMemcpyDeviceToHost, j->st);
    if (!rc && e == hipSuccess && j->desc.want_links)
      e = hipMemcpyAsync(j->hbase + j->lay.h_links, d + j->lay.canon, 4ull * j->g.V * 9 * 16,
                         hipMemcpyDeviceToHost, j->st);
    if (!rc && e == hipSuccess) e = hipEventCreateWithFlags(&j->done_ev, hipEventDisableTiming);
    if (!rc && e == hipSuccess) e = hipEventRecord(j->done_ev, j->st);
    if (!rc && e != hipSuccess) rc = note_hip_error(e);
    return rc;
  }

  // Admits queued jobs in FIFO order while the head fits.
  int admit() {
    while (!queue.empty() && !free_slots.empty()) {
      Job* j = queue.front();
      size_t doff, hoff;
      if (!dev_arena->alloc(j->lay.dev_total, &doff)) break;
      if (!host_arena->alloc(j->lay.host_total, &hoff)) {
        dev_arena->release(doff, j->lay.dev_total);
        break;
      }
      queue.pop_front();
      j->dev_off = doff;
      j->host_off = hoff;
      j->has_dev = j->has_host = true;
      j->dbase = dev_pool + doff;
      j->hbase = host_pool + hoff;
      j->slot = free_slots.back();
      free_slots.pop_back();
      j->state = VSM_JOB_RUNNING;
      j->t_admit = now();
      j->small = j->g.V <= kSmallSites;
      j->st = j->small ? stream_small : stream;
      (j->small ? running_small : running).push_back(j);
      hipStream_t st = j->st;
      const size_t V = j->g.V;
      char* d = j->dbase;
      memcpy(j->hbase + j->lay.h_in_z3, j->z3.data(), 4 * V);
      if (j->desc.pair_host) memcpy(j->hbase + j->lay.h_in_pairs, j->pairs.data(), 4 * V);
      std::vector<int8_t>().swap(j->z3);
      std::vector<int8_t>().swap(j->pairs);
      ServeJob sj;
      sj.g = j->g;
      sj.links = d + j->lay.links;
      sj.z3 = (const int8_t*)(d + j->lay.z3);
      sj.rej = (unsigned long long*)(d + j->lay.ws);
      sj.p = j->p;
      // the descriptor staging of a slot is reused only after the slot's
      // previous job has completed on the device
      desc_host[j->slot] = sj;
      hipError_t e = hipMemcpyAsync(jobs_dev + j->slot, desc_host + j->slot, sizeof(ServeJob),
                                    hipMemcpyHostToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(d + j->lay.z3, j->hbase + j->lay.h_in_z3, 4 * V, hipMemcpyHostToDevice, st);
      if (e == hipSuccess && j->desc.pair_host)
        e = hipMemcpyAsync(d + j->lay.pairs, j->hbase + j->lay.h_in_pairs, 4 * V, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return note_hip_error(e);
      if (j->desc.pair_host)
        launch_centrifuge(j->desc.precision, j->g, (const int8_t*)(d + j->lay.z3),
                          (const int8_t*)(d + j->lay.pairs), j->desc.omega, d + j->lay.links, nullptr, st);
      else
        launch_load_z3(j->desc.precision, j->g, (const int8_t*)(d + j->lay.z3), d + j->lay.links, st);
      launch_charges(j->g, (const int8_t*)(d + j->lay.z3),
                     (int8_t*)(d + j->lay.ws + ws_layout(j->desc.dims, j->desc.precision, VSM_ANNEALED).charges), 0,
                     4, st);
      launch_zero_u64((unsigned long long*)(d + j->lay.ws), 1, st);
      ctr.launches += 3;
      int rc = hip_status();
      if (rc) return rc;
      const int64_t resident = (int64_t)(running.size() + running_small.size() + finishing.size());
      if (resident > ctr.peak_resident_jobs) ctr.peak_resident_jobs = resident;
      if (j->n_pass == 0) {
        (j->small ? running_small : running).pop_back();
        rc = enqueue_finish(j);
        if (rc) return rc;
        finishing.push_back(j);
      }
    }
    ctr.peak_pool_bytes = dev_arena->peak();
    return VSM_OK;
  }

  // One scheduler step: the next pass of every running job.
  int step() {
    std::vector<Job*> order(running.begin(), running.end());
    for (int prec = 0; prec < 2; ++prec) {
      BatchStep bs;
      memset(&bs, 0, sizeof(bs));
      uint32_t nb = 0;
      auto flush = [&]() -> int {
        if (bs.njobs == 0) return VSM_OK;
        launch_update_batch(prec, jobs_dev, bs, nb, stream);
        ++ctr.launches;
        memset(&bs, 0, sizeof(bs));
        nb = 0;
        return hip_status();
      };
      for (Job* j : order) {
        if (j->desc.precision != prec) continue;
        const int64_t k = j->pass % 16;
        const int mu = (int)(k / 4);
        bs.first_block[bs.njobs] = nb;
        bs.slot[bs.njobs] = (uint32_t)j->slot;
        bs.mu[bs.njobs] = (uint8_t)j->g.perm[mu];
        bs.colour[bs.njobs] = (uint8_t)kColours[k % 4];
        ++bs.njobs;
        nb += pass_blocks(j->g);
        ctr.link_updates += j->g.V4;
        if (bs.njobs == (uint32_t)kBatchMax) {
          const int rc = flush();
          if (rc) return rc;
        }
      }
      const int rc = flush();
      if (rc) return rc;
    }
    // bookkeeping after the passes: records at sweep ends, and the end of jobs
    for (Job* j : order) {
      ++j->pass;
      if (j->pass % 16 == 0) {
        const int sw = (int)(j->pass / 16);
        if (j->desc.measure_every > 0 && sw % j->desc.measure_every == 0) {
          const int rc = enqueue_measure(j, sw);
          if (rc) return rc;
        }
      }
      if (j->pass == j->n_pass) {
        const int rc = enqueue_finish(j);
        if (rc) return rc;
      }
    }
    for (auto it = running.begin(); it != running.end();) {
      if ((*it)->pass == (*it)->n_pass) {
        finishing.push_back(*it);
        it = running.erase(it);
      } else {
        ++it;
      }
    }
    ++ctr.steps;
    return VSM_OK;
  }

  // One small-lattice step: every running small job advances by whole sweeps
  // inside one workgroup (k_serve_small), about kSmallStepSites sites' worth of
  // sweeps each, so that a step costs about the same for every job; a step
  // stops at the job's next measurement and at its last sweep.
  static constexpr int64_t kSmallStepSites = 32768;

  int small_step() {
    std::vector<Job*> order(running_small.begin(), running_small.end());
    std::vector<int> nsw(order.size(), 0);
    for (size_t i = 0; i < order.size(); ++i) {
      Job* j = order[i];
      const int done = (int)(j->pass / 16), total = j->desc.n_sweeps;
      int c = (int)(kSmallStepSites / (int64_t)j->g.V);
      if (c < 1) c = 1;
      if (c > total - done) c = total - done;
      const int me = j->desc.measure_every;
      if (me > 0 && c > me - done % me) c = me - done % me;
      nsw[i] = c;
    }
    for (int prec = 0; prec < 2; ++prec) {
      SmallStep ss;
      memset(&ss, 0, sizeof(ss));
      auto flush = [&]() -> int {
        if (ss.njobs == 0) return VSM_OK;
        launch_serve_small(prec, jobs_dev, ss, stream_small);
        ++ctr.launches;
        memset(&ss, 0, sizeof(ss));
        return hip_status();
      };
      for (size_t i = 0; i < order.size(); ++i) {
        Job* j = order[i];
        if (j->desc.precision != prec) continue;
        ss.slot[ss.njobs] = (uint16_t)j->slot;
        ss.sweeps[ss.njobs] = (uint16_t)nsw[i];
        ++ss.njobs;
        ctr.link_updates += 4ll * j->g.V * nsw[i];
        if (ss.njobs == (uint32_t)kSmallMax) {
          const int rc = flush();
          if (rc) return rc;
        }
      }
      const int rc = flush();
      if (rc) return rc;
    }
    for (size_t i = 0; i < order.size(); ++i) {
      Job* j = order[i];
      j->pass += 16ll * nsw[i];
      const int sw = (int)(j->pass / 16);
      if (j->desc.measure_every > 0 && sw % j->desc.measure_every == 0) {
        const int rc = enqueue_measure(j, sw);
        if (rc) return rc;
      }
      if (j->pass == j->n_pass) {
        const int rc = enqueue_finish(j);
        if (rc) return rc;
      }
    }
    for (auto it = running_small.begin(); it != running_small.end();) {
      if ((*it)->pass == (*it)->n_pass) {
        finishing.push_back(*it);
        it = running_small.erase(it);
      } else {
        ++it;
      }
    }
    ++ctr.steps;
    return VSM_OK;
  }

  // Moves finishing jobs whose results have reached the host to DONE.
  void retire() {
    for (auto it = finishing.begin(); it != finishing.end();) {
      Job* j = *it;
      const hipError_t e = hipEventQuery(j->done_ev);
      if (e == hipErrorNotReady) {
        ++it;
        continue;
      }
      if (e == hipSuccess) {
        j->state = VSM_JOB_DONE;
        j->t_done = now();
        ++ctr.jobs_done;
      } else {
        fail_job(j, note_hip_error(e));
      }
      release_device(j);
      it = finishing.erase(it);
      cv_done.notify_all();
    }
  }

  void break_all(int rc) {
    broken = rc;
    (void)hipStreamSynchronize(stream);
    (void)hipStreamSynchronize(stream_small);
    for (Job* j : running) {
      fail_job(j, rc);
      release_device(j);
    }
    running.clear();
    for (Job* j : running_small) {
      fail_job(j, rc);
      release_device(j);
    }
    running_small.clear();
    for (Job* j : finishing) {
      fail_job(j, rc);
      release_device(j);
    }
    finishing.clear();
    for (Job* j : queue) fail_job(j, rc);
    queue.clear();
    cv_done.notify_all();
  }

  void run() {
    std::unique_lock<std::mutex> lk(mu);
    {
      const hipError_t e = hipSetDevice(cfg.device);
      if (e != hipSuccess) break_all(note_hip_error(e));
    }
    int64_t nstep = 0, nsmall = 0;
    double busy_from = -1;
    // a stream may take its next step when fewer than max_inflight of its steps
    // are still queued on the device (*err: a failed query)
    auto room = [&](const std::vector<hipEvent_t>& ev, int64_t n, int* err) -> bool {
      *err = VSM_OK;
      if (n < cfg.max_inflight) return true;
      const hipError_t e = hipEventQuery(ev[n % cfg.max_inflight]);
      if (e == hipErrorNotReady) return false;
      if (e != hipSuccess) *err = note_hip_error(e);
      return e == hipSuccess;
    };
    for (;;) {
      const uint64_t seen = gen;
      retire();
      if (!stopping && !broken) {
        const int rc = admit();
        if (rc) {
          break_all(rc);
          continue;
        }
      }
      const bool resident = !running.empty() || !running_small.empty() || !finishing.empty();
      if (resident && busy_from < 0) busy_from = now();
      if (!resident && busy_from >= 0) {
        ctr.busy_seconds += now() - busy_from;
        busy_from = -1;
      }
      if (running.empty() && running_small.empty()) {
        if (!finishing.empty()) {
          hipEvent_t ev = finishing.front()->done_ev;
          lk.unlock();
          const hipError_t e = hipEventSynchronize(ev);
          lk.lock();
          if (e != hipSuccess) break_all(note_hip_error(e));
          continue;
        }
        if (stopping) break;
        cv_work.wait(lk, [&] { return stopping || gen != seen; });
        continue;
      }
      if (stopping) break;
      bool progressed = false;
      int err = VSM_OK;
      if (!running.empty()) {
        const bool r = room(step_ev, nstep, &err);
        if (err) {
          break_all(err);
          continue;
        }
        if (r) {
          int rc = step();
          if (!rc) rc = note_hip_error(hipEventRecord(step_ev[nstep % cfg.max_inflight], stream));
          if (rc) {
            break_all(rc);
            continue;
          }
          ++nstep;
          progressed = true;
        }
      }
      if (!running_small.empty()) {
        const bool r = room(small_ev, nsmall, &err);
        if (err) {
          break_all(err);
          continue;
        }
        if (r) {
          int rc = small_step();
          if (!rc) rc = note_hip_error(hipEventRecord(small_ev[nsmall % cfg.max_inflight], stream_small));
          if (rc) {
            break_all(rc);
            continue;
          }
          ++nsmall;
          progressed = true;
        }
      }
      if (!progressed) {
        // both streams have max_inflight steps queued: let the device catch up
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      }
    }
    if (busy_from >= 0) ctr.busy_seconds += now() - busy_from;
    // shutdown: let the device finish, keep what completed, fail the rest
    lk.unlock();
    (void)hipStreamSynchronize(stream);
    (void)hipStreamSynchronize(stream_small);
    lk.lock();
    retire();
    for (Job* j : finishing) {
      fail_job(j, VSM_E_STATE);
      release_device(j);
    }
    finishing.clear();
    for (Job* j : running) {
      fail_job(j, VSM_E_STATE);
      release_device(j);
    }
    running.clear();
    for (Job* j : running_small) {
      fail_job(j, VSM_E_STATE);
      release_device(j);
    }
    running_small.clear();
    for (Job* j : queue) fail_job(j, VSM_E_STATE);
    queue.clear();
    cv_done.notify_all();
  }

  void fill_info(const Job* j, vsm_job_info* info) const {
    info->state = j->state;
    info->status = j->status;
    info->n_records = j->n_records;
    info->sweeps_done = (int32_t)(j->pass / 16);
    info->t_submit = j->t_submit;
    info->t_admit = j->t_admit;
    info->t_done = j->t_done;
    info->footprint_bytes = j->lay.dev_total;
  }
};

void free_server(Server* s) {
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->stream_small) (void)hipStreamSynchronize(s->stream_small);
  for (hipEvent_t e : s->step_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : s->small_ev) (void)hipEventDestroy(e);
  for (auto& kv : s->jobs)
    if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
  if (s->dev_pool) (void)hipFree(s->dev_pool);
  if (s->jobs_dev) (void)hipFree(s->jobs_dev);
  if (s->host_pool) (void)hipHostFree(s->host_pool);
  if (s->desc_host) (void)hipHostFree(s->desc_host);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->stream_small) (void)hipStreamDestroy(s->stream_small);
  delete s;
}

}  // namespace

extern "C" {

size_t vsm_server_job_bytes(const vsm_job* job) {
  if (validate_job(job) != VSM_OK) return 0;
  return layout_of(*job).dev_total;
}

size_t vsm_server_host_bytes(const vsm_job* job) {
  if (validate_job(job) != VSM_OK) return 0;
  return layout_of(*job).host_total;
}

int vsm_server_create(const vsm_server_config* cfg, void** srv) {
  if (!cfg || !srv) return VSM_E_NULL;
  *srv = nullptr;
  if (cfg->hbm_budget_bytes == 0 || cfg->host_budget_bytes == 0 || cfg->max_slots < 1 ||
      cfg->max_slots > 256 || cfg->max_inflight < 1 || cfg->max_inflight > 64 || cfg->device < 0)
    return VSM_E_PARAM;
  Server* s = new Server();
  s->cfg = *cfg;
  s->t0 = std::chrono::steady_clock::now();
  hipError_t e = hipSetDevice(cfg->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream_small, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc((void**)&s->dev_pool, cfg->hbm_budget_bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&s->jobs_dev, sizeof(ServeJob) * (size_t)cfg->max_slots);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->host_pool, cfg->host_budget_bytes, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&s->desc_host, sizeof(ServeJob) * (size_t)cfg->max_slots, hipHostMallocDefault);
  for (int i = 0; e == hipSuccess && i < cfg->max_inflight; ++i) {
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) s->step_ev.push_back(ev);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) s->small_ev.push_back(ev);
  }
  if (e != hipSuccess) {
    const int rc = note_hip_error(e);
    free_server(s);
    return rc;
  }
  s->dev_arena.reset(new Arena(cfg->hbm_budget_bytes));
  s->host_arena.reset(new Arena(cfg->host_budget_bytes));
  for (int i = cfg->max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  s->worker = std::thread([s] { s->run(); });
  *srv = s;
  return VSM_OK;
}

int vsm_server_submit(void* srv, const vsm_job* job, uint64_t* job_id) {
  Server* s = (Server*)srv;
  if (!s || !job_id) return VSM_E_NULL;
  int rc = validate_job(job);
  if (rc) return rc;
  const JobLayout lay = layout_of(*job);
  if (lay.dev_total > s->cfg.hbm_budget_bytes || lay.host_total > s->cfg.host_budget_bytes)
    return VSM_E_BUDGET;
  std::unique_ptr<Job> j(new Job());
  j->desc = *job;
  j->g = make_geo(job->dims);
  j->p = make_params(job->rho, job->eps, &job->sched);
  j->lay = lay;
  j->n_records = n_records_of(*job);
  j->n_pass = 16ll * job->n_sweeps;
  const size_t V = j->g.V;
  j->z3.assign(job->z3_host, job->z3_host + 4 * V);
  if (job->pair_host) j->pairs.assign(job->pair_host, job->pair_host + 4 * V);
  j->desc.z3_host = nullptr;
  // from here on desc.pair_host only says whether the job has pairs
  j->desc.pair_host = job->pair_host ? (const int8_t*)j->pairs.data() : nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return VSM_E_STATE;
  if (s->broken) return s->broken;
  j->id = s->next_id++;
  j->t_submit = s->now();
  *job_id = j->id;
  s->queue.push_back(j.get());
  s->jobs.emplace(j->id, std::move(j));
  ++s->ctr.jobs_submitted;
  ++s->gen;
  s->cv_work.notify_all();
  return VSM_OK;
}

int vsm_server_poll(void* srv, uint64_t job_id, vsm_job_info* info) {
  Server* s = (Server*)srv;
  if (!s || !info) return VSM_E_NULL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return VSM_E_STATE;
  s->fill_info(it->second.get(), info);
  return VSM_OK;
}

int vsm_server_wait(void* srv, uint64_t job_id, double timeout_s, vsm_job_info* info) {
  Server* s = (Server*)srv;
  if (!s || !info) return VSM_E_NULL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return VSM_E_STATE;
  Job* j = it->second.get();
  auto finished = [&] { return j->state == VSM_JOB_DONE || j->state == VSM_JOB_FAILED; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, finished);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished)) {
    s->fill_info(j, info);
    return VSM_E_TIMEOUT;
  }
  s->fill_info(j, info);
  return VSM_OK;
}

int vsm_server_fetch(void* srv, uint64_t job_id, vsm_stats* records_host, int32_t max_records,
                     double* links_host) {
  Server* s = (Server*)srv;
  if (!s) return VSM_E_NULL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return VSM_E_STATE;
  Job* j = it->second.get();
  if (j->state != VSM_JOB_DONE && j->state != VSM_JOB_FAILED) return VSM_E_STATE;
  int rc = j->status;
  if (j->state == VSM_JOB_DONE) {
    if (max_records > 0 && !records_host) return VSM_E_NULL;
    const int n = max_records < j->n_records ? (max_records < 0 ? 0 : max_records) : j->n_records;
    if (n > 0) memcpy(records_host, j->hbase + j->lay.h_records, (size_t)n * sizeof(vsm_stats));
    if (links_host) {
      if (!j->desc.want_links) return VSM_E_STATE;
      memcpy(links_host, j->hbase + j->lay.h_links, 4ull * j->g.V * 9 * 16);
    }
    rc = VSM_OK;
  }
  if (j->has_host) s->host_arena->release(j->host_off, j->lay.host_total);
  j->has_host = false;
  s->jobs.erase(it);
  ++s->gen;
  s->cv_work.notify_all();  // freed host pool may let the queue head in
  return rc;
}

double vsm_server_clock(void* srv) {
  Server* s = (Server*)srv;
  return s ? s->now() : -1.0;
}

int vsm_server_get_counters(void* srv, vsm_server_counters* out) {
  Server* s = (Server*)srv;
  if (!s || !out) return VSM_E_NULL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->ctr;
  return VSM_OK;
}

int vsm_server_destroy(void* srv) {
  Server* s = (Server*)srv;
  if (!s) return VSM_E_NULL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  free_server(s);
  return VSM_OK;
}

}  // extern "C"
