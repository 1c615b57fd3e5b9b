// tune_cache.hpp -- choices of the autotuners (linear plans, RK plans, the
// batched server's z-march depths), keyed by shape class (internal).
//
// Process-wide map from a key string to a few integers. If the environment
// variable STENCIL_TUNE_CACHE names a file, it is read once on first use
// (lines "key v0 v1 ...") and every new choice is appended to it, so a later
// process starts from the choices an earlier one measured.
#pragma once

#include <string>
#include <vector>

namespace stn {

bool tune_cache_get(const std::string &key, std::vector<int> &vals);
void tune_cache_put(const std::string &key, const std::vector<int> &vals);

} // namespace stn
