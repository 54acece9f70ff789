// Host-side brick map of a voxel box (see ep_internal.h for the layout):
// active 8x8x8 bricks in x-major brick order, the ghost brick, the 27-entry
// neighbour table and the tissue mask in brick layout.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "ep_internal.h"

namespace ep {

struct BrickMap {
  int n[3] = {0, 0, 0};
  int nbx = 0, nby = 0, nbz = 0, nb = 0;
  int64_t n_tissue = 0;
  int64_t nvox = 0;            // (nb + 1) * 512, ghost included
  std::vector<int> brick_id;   // nbx*nby*nbz -> id or -1
  std::vector<int> brick_pos;  // id -> (bx, by, bz)
  std::vector<int> nbr;        // (nb + 1) * 27, ghost = nb
  std::vector<uint8_t> mask;   // nvox, brick layout

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
  int64_t tissue = 0;
  for (int x = 0; x < n[0]; ++x)
    for (int y = 0; y < n[1]; ++y)
      for (int z = 0; z < n[2]; ++z)
        if (!boxmask || boxmask[m.box_index(x, y, z)]) {
          ++tissue;
          m.brick_id[(static_cast<int64_t>(x >> 3) * m.nby + (y >> 3)) * m.nbz + (z >> 3)] = 0;
        }
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
  for (int id = 0; id < nb; ++id) {
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
  }
  m.mask.assign(m.nvox, 0);
  for (int x = 0; x < n[0]; ++x)
    for (int y = 0; y < n[1]; ++y)
      for (int z = 0; z < n[2]; ++z)
        if (!boxmask || boxmask[m.box_index(x, y, z)]) m.mask[m.brick_index(x, y, z)] = 1;
  return true;
}

}  // namespace ep
