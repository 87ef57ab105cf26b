// Host-side internals shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/gabm.h"
#include "gabm_device.h"

namespace gabm {

void set_error(const std::string& msg);

// RAII-free device buffer helpers (the library frees explicitly).
template <typename T>
inline hipError_t dalloc(T** p, size_t n) {
  if (n == 0) n = 1;
  return hipMalloc((void**)p, n * sizeof(T));
}

struct Graph {
  int32_t N = 0, n_pops = 0, n_age = 0;
  int64_t E = 0;
  int32_t max_degree = 0, n_tiles = 0, n_long = 0;
  double weight_sum = 0.0;
  std::vector<int32_t> pop_off_h;   // [n_pops+1]
  std::vector<int64_t> er_off_h;    // [n_pops+1]
  float er_mean = 0.f, er_w = 0.f;
  // device
  int64_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  float* w = nullptr;
  int32_t* tile_row = nullptr;
  TileInfo* tiles = nullptr;
  TileInfo* btiles = nullptr;
  int32_t n_btiles = 0;
  uint32_t* colp = nullptr;
  float* wp = nullptr;
  uint32_t* chunk_row = nullptr;
  int64_t n_chunks = 0;  // 0 = edge-parallel form not available
  // sender-sliced stream of the split B = 1 kernels (packed like colp / wp,
  // one receiver-sorted stream per slice, each starting at a chunk
  // boundary); n_slices = 0 when not built
  uint32_t* fcolp = nullptr;
  float* fwp = nullptr;
  unsigned long long* fchunk_hdr = nullptr;  // chunk headers (see the split kernels)
  int32_t n_slices = 0;
  std::vector<int64_t> slice_chunk;  // [n_slices + 1] first chunk of each slice; last = chunk count
  uint8_t* age = nullptr;
  uint16_t* pop_of = nullptr;
  int32_t* pop_off = nullptr;
  int64_t* er_off = nullptr;
  // agent-location layer: visits sorted by location (stable in input order)
  // and by agent; n_visits = 0 when the graph has none
  int32_t n_loc = 0;
  int64_t n_visits = 0;
  int32_t* lv_agent = nullptr;  // [V] visitor of each location-sorted visit
  int32_t* lv_loc = nullptr;    // [V] its location (runs of equal ids)
  float* lv_w = nullptr;        // [V]
  int64_t* av_ptr = nullptr;    // [N+1] visits of agent i: av_ptr[i] .. av_ptr[i+1]
  int32_t* av_loc = nullptr;    // [V]
  float* av_w = nullptr;        // [V]
  double* loc_scratch = nullptr;  // [2 * n_loc] pressures of the single-step sums
  bool has_er() const { return !er_off_h.empty() && er_off_h.back() > 0; }
  // a layer whose sums arrive through the per-agent accumulators (daily random
  // pairs, or locations)
  bool has_aux() const { return has_er() || n_visits > 0; }

  DGraph view() const {
    DGraph g;
    g.row_ptr = row_ptr; g.col = col; g.w = w; g.tile_row = tile_row; g.tiles = tiles; g.btiles = btiles; g.n_btiles = n_btiles; g.age = age;
    g.colp = colp; g.wp = wp; g.chunk_row = chunk_row; g.n_chunks = n_chunks; g.pop_of = pop_of;
    g.pop_off = pop_off; g.er_off = er_off; g.N = N; g.n_pops = n_pops; g.n_tiles = n_tiles;
    g.er_total = er_off_h.empty() ? 0 : er_off_h.back();
    g.er_mean = er_mean; g.er_w = er_w;
    return g;
  }
  void release();
};

// checks the parameter block against the graph; fills `out` (kernel view)
gabm_status check_params(const Graph& G, const gabm_params* p, DParams* out);

#define GABM_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      ::gabm::set_error(std::string(#call) + ": " + hipGetErrorString(e_));   \
      return GABM_EHIP;                                                       \
    }                                                                         \
  } while (0)

#define GABM_CHECK(cond, code, msg) \
  do {                              \
    if (!(cond)) {                  \
      ::gabm::set_error(msg);       \
      return code;                  \
    }                               \
  } while (0)

}  // namespace gabm

struct gabm_graph_s {
  gabm::Graph g;
};
