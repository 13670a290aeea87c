// Optional per-kernel timing with HIP events on the launch stream.
//
// When a context enables timing, every launcher brackets its kernel with two
// events (only for kernels whose name passes the filter) and records the
// algorithmic bytes of that launch: the bytes the kernel must read and write
// at minimum (each operand once).  flush() waits for the events and adds
// the durations to per-kernel totals.
//
// Filter: empty (every kernel), a kernel name, "name@l" (that kernel's
// launches on level l only), or "@" (every kernel, totals kept per level
// under the name "name@l" for launchers that state their level).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

namespace cmg {

struct KernelTiming {
  struct Pending {
    int id;
    double bytes;
    hipEvent_t a, b;
  };
  std::string filter;  // empty: every kernel; otherwise one kernel name
  std::vector<std::string> names;
  std::vector<long long> launches;
  std::vector<double> ms, bytes;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipStream_t st = nullptr;
  int open = -1;

  int id_of(const char* name) {
    for (size_t i = 0; i < names.size(); ++i)
      if (names[i] == name) return static_cast<int>(i);
    names.emplace_back(name);
    launches.push_back(0);
    ms.push_back(0.0);
    bytes.push_back(0.0);
    return static_cast<int>(names.size() - 1);
  }
  hipEvent_t next_event() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(const char* name, double nbytes, hipStream_t s, int level = -1) {
    open = -1;
    std::string key = name;
    if (filter == "@") {
      if (level >= 0) key += "@" + std::to_string(level);
    } else if (!filter.empty()) {
      const size_t at = filter.find('@');
      if (at == std::string::npos ? filter != key
                                  : (filter.compare(0, at, key) != 0 || at != key.size() ||
                                     filter.substr(at + 1) != std::to_string(level)))
        return;
    }
    hipEvent_t a = next_event(), b = next_event();
    if (a == nullptr || b == nullptr) return;
    (void)hipEventRecord(a, s);
    pending.push_back(Pending{id_of(key.c_str()), nbytes, a, b});
    open = static_cast<int>(pending.size() - 1);
    st = s;
  }
  void end(hipStream_t s) {
    if (open < 0) return;
    (void)hipEventRecord(pending[open].b, s);
    open = -1;
  }
  void flush() {
    for (const Pending& p : pending) {
      float t = 0.f;
      (void)hipEventSynchronize(p.b);
      (void)hipEventElapsedTime(&t, p.a, p.b);
      launches[p.id] += 1;
      ms[p.id] += t;
      bytes[p.id] += p.bytes;
    }
    pending.clear();
    used = 0;
  }
  void reset() {
    flush();
    names.clear();
    launches.clear();
    ms.clear();
    bytes.clear();
  }
  ~KernelTiming() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// The sink of the context whose call is running on this thread (or null).
extern thread_local KernelTiming* g_timing;

}  // namespace cmg
