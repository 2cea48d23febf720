// Optional per-kernel timing with HIP events recorded on the launch stream.
// Disabled by default; when enabled, named kernel launches are bracketed by
// event pairs that are resolved (summed) when read.
#pragma once

#include <hip/hip_runtime.h>

namespace yr {

bool prof_on();
// returns an opaque slot (or -1 when disabled); call prof_end with it
int prof_begin(const char* name, hipStream_t s);
void prof_end(int slot, hipStream_t s);

struct ProfScope {
  int slot;
  hipStream_t s;
  ProfScope(const char* name, hipStream_t st) : slot(prof_on() ? prof_begin(name, st) : -1), s(st) {}
  ~ProfScope() {
    if (slot >= 0) prof_end(slot, s);
  }
};

}  // namespace yr
