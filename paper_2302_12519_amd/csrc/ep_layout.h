// Host-side brick map of a voxel box (see ep_internal.h for the layout):
// active 8x8x8 bricks in x-major brick order, the ghost brick, the 27-entry
// neighbour table and the tissue mask in brick layout.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "ep_internal.h"

namespace ep {

// Run f(i) for every i in [0, n) on up to 16 host threads, in contiguous
// chunks.  f must not throw and must touch disjoint data for distinct i.
template <typename F>
void parallel_for(int64_t n, F&& f) {
  const int64_t hw = std::max<int64_t>(1, std::thread::hardware_concurrency());
  const int64_t nt = std::min<int64_t>({16, hw, n});
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(static_cast<size_t>(nt));
  const int64_t chunk = (n + nt - 1) / nt;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([&f, lo, hi] {
      for (int64_t i = lo; i < hi; ++i) f(i);
    });
  }
  for (auto& x : th) x.join();
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
  // tissue count and brick occupancy, one x-slab of bricks per task
  std::vector<int64_t> slab_tissue(m.nbx, 0);
  parallel_for(m.nbx, [&](int64_t bx) {
    int64_t t = 0;
    for (int x = static_cast<int>(8 * bx); x < std::min(n[0], static_cast<int>(8 * bx + 8)); ++x)
      for (int y = 0; y < n[1]; ++y)
        for (int z = 0; z < n[2]; ++z)
          if (!boxmask || boxmask[m.box_index(x, y, z)]) {
            ++t;
            m.brick_id[(bx * m.nby + (y >> 3)) * m.nbz + (z >> 3)] = 0;
          }
    slab_tissue[bx] = t;
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
  m.mask.assign(m.nvox, 0);
  parallel_for(m.nbx, [&](int64_t bx) {
    for (int x = static_cast<int>(8 * bx); x < std::min(n[0], static_cast<int>(8 * bx + 8)); ++x)
      for (int y = 0; y < n[1]; ++y)
        for (int z = 0; z < n[2]; ++z)
          if (!boxmask || boxmask[m.box_index(x, y, z)]) m.mask[m.brick_index(x, y, z)] = 1;
  });
  m.rows.assign(nb + 1, 0);
  parallel_for(nb, [&](int64_t id) {
    uint64_t r = 0;
    for (int l = 0; l < kBV; ++l)
      if (m.mask[static_cast<size_t>(id) * kBV + l]) r |= uint64_t(1) << (l >> 3);
    m.rows[id] = r;
  });
  m.rowsn.assign(static_cast<size_t>(nb + 1) * kNbr, 0);
  for (size_t k = 0; k < m.rowsn.size(); ++k) m.rowsn[k] = m.rows[m.nbr[k]];
  return true;
}

}  // namespace ep
