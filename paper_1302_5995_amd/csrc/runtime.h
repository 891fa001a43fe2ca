// Internals of the runtime shared with the serving layer (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/dtn.h"

struct dtn_op {
  int device = 0;
  int n = 0, nb = 0, leaf = 0;
  double* T = nullptr;              // nb x nb, column-major, owned (device caching allocator)
  dtn_stats stats{};
  // split-K apply partial sums (allocated on the first narrow apply); applies of this handle on
  // different streams are ordered through part_ev so they never share the buffer concurrently
  double* part = nullptr;
  hipEvent_t part_ev = nullptr;
  bool part_ev_recorded = false;
  std::mutex part_mu;
};

namespace dtn {

void set_err(const std::string& s);
const std::string& last_err();
int device_ready(int dev);
void* dev_alloc(int dev, size_t bytes);
void dev_release(int dev, void* p);
// Device bytes the plan of (n, leaf, conv, fast) holds; resident = already cached on dev.
int plan_footprint(int dev, int n, int leaf, int conv, bool fast, size_t& bytes, bool& resident);

}  // namespace dtn
