// Internal definition of a cloud handle, shared by the host and device translation units.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "delaunay.h"
#include "mknn.h"

struct mknn_cloud {
  int64_t n = 0;
  std::vector<float> xyz;          // n x 3 float32 by rank
  std::vector<int32_t> order;      // rank -> caller id
  mknn::Csr succ;                  // successor lists (ranks ascending)
  mknn::Csr pred;                  // Delaunay neighbours at insertion (transpose of succ)
  std::vector<uint8_t> live;       // 1 = present
  int32_t head = 0;                // smallest live rank
  int64_t nlive = 0;
  float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};   // bounding box of all points
  uint64_t version = 0;            // bumped by every mutation

  // device residency
  int device = -1;
  void *d_ent = nullptr;           // 16-byte records {x, y, z, rank}, padded
  uint64_t *d_lst = nullptr;       // per rank: start | (length << 32)
  int64_t dev_bytes = 0;
  uint64_t dev_version = ~0ull;
};

namespace mknn {
mknn_status set_error(mknn_status s, const std::string &msg);
void clear_error();
}  // namespace mknn
