// Host-side brick map of a voxel box (see ep_internal.h for the layout):
// active 8x8x8 bricks in x-major brick order, the ghost brick, the 27-entry
// neighbour table and the tissue mask in brick layout.
#pragma once

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ep_internal.h"

namespace ep {

// A fixed pool of host worker threads, started on first use and kept for
// the life of the process, so that the many small parallel loops of grid
// creation and request submission do not each pay for starting threads.
// One loop runs on the pool at a time; a caller that finds it busy (another
// thread's loop) runs its loop serially instead of waiting.
class HostPool {
 public:
  static HostPool& get() {
    static HostPool p;
    return p;
  }
  int size() const { return static_cast<int>(workers_.size()) + 1; }
  // false if the pool is busy; otherwise runs body(t) for t in [0, nt) on
  // the workers and the caller and returns when all are done
  template <typename B>
  bool run(int nt, B& body) {
    std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
    if (!busy.owns_lock()) return false;
    {
      std::lock_guard<std::mutex> lk(mu_);
      call_ = [](void* b, int t) { (*static_cast<B*>(b))(t); };
      arg_ = &body;
      tasks_ = nt;
      next_.store(1);            // task 0 is the caller's
      left_ = static_cast<int>(workers_.size());
      ++gen_;
    }
    cv_.notify_all();
    body(0);
    for (int t; (t = next_.fetch_add(1)) < nt;) body(t);
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return left_ == 0; });
    return true;
  }

 private:
  HostPool() {
    const int hw = static_cast<int>(std::max(1u, std::thread::hardware_concurrency()));
    const int nw = std::min(16, hw) - 1;
    for (int k = 0; k < nw; ++k) workers_.emplace_back([this] { loop(); });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& w : workers_) w.join();
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
      if (stop_) return;
      seen = gen_;
      void (*call)(void*, int) = call_;
      void* arg = arg_;
      const int nt = tasks_;
      lk.unlock();
      for (int t; (t = next_.fetch_add(1)) < nt;) call(arg, t);
      lk.lock();
      if (--left_ == 0) done_cv_.notify_one();
    }
  }
  std::vector<std::thread> workers_;
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  void (*call_)(void*, int) = nullptr;
  void* arg_ = nullptr;
  int tasks_ = 0, left_ = 0;
  uint64_t gen_ = 0;
  std::atomic<int> next_{0};
  bool stop_ = false;
};

// Run f(i) for every i in [0, n) on the host pool (up to 16 threads), in
// contiguous chunks.  f must not throw and must touch disjoint data for
// distinct i.
template <typename F>
void parallel_for(int64_t n, F&& f) {
  HostPool& pool = HostPool::get();
  const int64_t nt = std::min<int64_t>(pool.size(), n);
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  const int64_t chunk = (n + nt - 1) / nt;
  auto body = [&f, n, chunk](int t) {
    const int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
    for (int64_t i = lo; i < hi; ++i) f(i);
  };
  if (!pool.run(static_cast<int>(nt), body))
    for (int64_t i = 0; i < n; ++i) f(i);
}

struct BrickMap {
  int n[3] = {0, 0, 0};
  int nbx = 0, nby = 0, nbz = 0, nb = 0;
  int64_t n_tissue = 0;
  int64_t nvox = 0;            // (nb + 1) * 512, ghost included
  std::vector<int> brick_id;   // nbx*nby*nbz -> id or -1
  std::vector<int> brick_pos;  // id -> (bx, by, bz)
  std::vector<int> nbr;        // (nb + 1) * 27, ghost = nb
  std::vector<uint8_t> mask;   // nvox, brick layout
  std::vector<uint64_t> rows;  // nb + 1: bit lx*8+ly set when row (lx, ly, *) holds tissue
  std::vector<uint64_t> rowsn; // (nb + 1) * 27: rows of each brick's neighbours (nbr order)

  int64_t box_index(int x, int y, int z) const {
    return (static_cast<int64_t>(x) * n[1] + y) * n[2] + z;
  }
  // brick-layout index of box voxel (x, y, z), or -1 if its brick is absent
  int64_t brick_index(int x, int y, int z) const {
    const int id = brick_id[(static_cast<int64_t>(x >> 3) * nby + (y >> 3)) * nbz + (z >> 3)];
    if (id < 0) return -1;
    return static_cast<int64_t>(id) * kBV + (((x & 7) * 8 + (y & 7)) * 8 + (z & 7));
  }
};

// Build the map of box n with tissue mask (box layout, nonzero = tissue;
// NULL = all tissue).  Returns false with a message when the mask holds no
// tissue or the brick count exceeds 32-bit indexing.
inline bool build_brick_map(const int n[3], const uint8_t* boxmask, BrickMap& m,
                            std::string& err) {
  for (int k = 0; k < 3; ++k) m.n[k] = n[k];
  m.nbx = (n[0] + 7) / 8;
  m.nby = (n[1] + 7) / 8;
  m.nbz = (n[2] + 7) / 8;
  const int64_t NB = static_cast<int64_t>(m.nbx) * m.nby * m.nbz;
  m.brick_id.assign(NB, -1);
  // tissue count and brick occupancy, one (x, y) column of bricks per task;
  // a brick row (8 voxels along z) is tested as one 64-bit word
  const int64_t ncol = static_cast<int64_t>(m.nbx) * m.nby;
  std::vector<int64_t> slab_tissue(ncol, 0);
  parallel_for(ncol, [&](int64_t col) {
    const int bx = static_cast<int>(col / m.nby), by = static_cast<int>(col % m.nby);
    int64_t t = 0;
    for (int x = 8 * bx; x < std::min(n[0], 8 * bx + 8); ++x)
      for (int y = 8 * by; y < std::min(n[1], 8 * by + 8); ++y) {
        if (!boxmask) {
          t += n[2];
          for (int bz = 0; bz < m.nbz; ++bz) m.brick_id[col * m.nbz + bz] = 0;
          continue;
        }
        const uint8_t* row = boxmask + m.box_index(x, y, 0);
        for (int z0 = 0; z0 < n[2]; z0 += 8) {
          const int len = std::min(8, n[2] - z0);
          uint64_t word = 0;
          std::memcpy(&word, row + z0, static_cast<size_t>(len));
          if (!word) continue;
          for (int z = 0; z < len; ++z) t += row[z0 + z] != 0;
          m.brick_id[col * m.nbz + (z0 >> 3)] = 0;
        }
      }
    slab_tissue[col] = t;
  });
  int64_t tissue = 0;
  for (int64_t t : slab_tissue) tissue += t;
  if (tissue == 0) {
    err = "mask holds no tissue";
    return false;
  }
  int nb = 0;
  m.brick_pos.clear();
  for (int64_t b = 0; b < NB; ++b)
    if (m.brick_id[b] >= 0) {
      m.brick_id[b] = nb++;
      m.brick_pos.push_back(static_cast<int>(b / (static_cast<int64_t>(m.nby) * m.nbz)));
      m.brick_pos.push_back(static_cast<int>((b / m.nbz) % m.nby));
      m.brick_pos.push_back(static_cast<int>(b % m.nbz));
    }
  if (static_cast<int64_t>(nb + 1) * kBV >= (int64_t(1) << 31)) {
    err = "grid too large for 32-bit brick indexing";
    return false;
  }
  m.nb = nb;
  m.n_tissue = tissue;
  m.nvox = static_cast<int64_t>(nb + 1) * kBV;
  m.nbr.assign(static_cast<size_t>(nb + 1) * kNbr, nb);
  parallel_for(nb, [&](int64_t id) {
    const int bx = m.brick_pos[3 * id], by = m.brick_pos[3 * id + 1], bz = m.brick_pos[3 * id + 2];
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          const int x = bx + dx, y = by + dy, z = bz + dz;
          int v = nb;
          if (x >= 0 && y >= 0 && z >= 0 && x < m.nbx && y < m.nby && z < m.nbz) {
            const int id2 = m.brick_id[(static_cast<int64_t>(x) * m.nby + y) * m.nbz + z];
            if (id2 >= 0) v = id2;
          }
          m.nbr[static_cast<size_t>(id) * kNbr + (dx + 1) * 9 + (dy + 1) * 3 + (dz + 1)] = v;
        }
  });
  // the mask in brick layout and each brick's row mask, one brick per task
  m.mask.assign(m.nvox, 0);
  m.rows.assign(nb + 1, 0);
  parallel_for(nb, [&](int64_t id) {
    const int bx = m.brick_pos[3 * id], by = m.brick_pos[3 * id + 1], bz = m.brick_pos[3 * id + 2];
    uint8_t* out = m.mask.data() + static_cast<size_t>(id) * kBV;
    uint64_t r = 0;
    for (int lx = 0; lx < 8; ++lx)
      for (int ly = 0; ly < 8; ++ly) {
        const int x = 8 * bx + lx, y = 8 * by + ly;
        if (x >= n[0] || y >= n[1]) continue;
        bool any = false;
        for (int lz = 0; lz < 8; ++lz) {
          const int z = 8 * bz + lz;
          if (z >= n[2]) break;
          const bool t = !boxmask || boxmask[m.box_index(x, y, z)];
          out[(lx * 8 + ly) * 8 + lz] = t ? 1 : 0;
          any = any || t;
        }
        if (any) r |= uint64_t(1) << (lx * 8 + ly);
      }
    m.rows[id] = r;
  });
  m.rowsn.assign(static_cast<size_t>(nb + 1) * kNbr, 0);
  for (size_t k = 0; k < m.rowsn.size(); ++k) m.rowsn[k] = m.rows[m.nbr[k]];
  return true;
}

}  // namespace ep
