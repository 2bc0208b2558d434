// Kernel-plan cache of the setup autotuner: a text file of "key value" lines,
// one per tuned shape.  The key names the device (architecture and compute
// units), the kernel class, the precision and the shape; the value is the
// plan the timing chose ("plan=1 blocks=1024", ...).  A setup that finds its
// key skips the timing; one that times appends its result.  A missing or
// unreadable file behaves as an empty cache; a file that cannot be written
// leaves the tuned plan in force for the handle only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

namespace bltt {
namespace plans {

inline std::mutex& file_mutex() {
  static std::mutex m;
  return m;
}

// architecture name and compute-unit count of the current device
inline std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  return arch + "/cu" + std::to_string(prop.multiProcessorCount);
}

// the last value stored for `key` (later lines override earlier ones)
inline bool lookup(const std::string& path, const std::string& key, std::string* value) {
  if (path.empty()) return false;
  std::lock_guard<std::mutex> lock(file_mutex());
  std::ifstream in(path);
  if (!in) return false;
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    if (line.size() > key.size() && line.compare(0, key.size(), key) == 0 && line[key.size()] == '\t') {
      *value = line.substr(key.size() + 1);
      found = true;
    }
  }
  return found;
}

inline void store(const std::string& path, const std::string& key, const std::string& value) {
  if (path.empty()) return;
  std::lock_guard<std::mutex> lock(file_mutex());
  std::ofstream out(path, std::ios::app);
  if (out) out << key << '\t' << value << '\n';
}

// "name=int" fields of a stored value
inline std::map<std::string, long> fields(const std::string& value) {
  std::map<std::string, long> f;
  std::istringstream is(value);
  std::string tok;
  while (is >> tok) {
    const size_t eq = tok.find('=');
    if (eq == std::string::npos) continue;
    char* end = nullptr;
    const long v = std::strtol(tok.c_str() + eq + 1, &end, 10);
    if (end && *end == '\0') f[tok.substr(0, eq)] = v;
  }
  return f;
}

}  // namespace plans
}  // namespace bltt
