// Optional per-kernel timing with HIP events (off unless sched_profile(1)).
#pragma once

#include <hip/hip_runtime.h>

namespace schedk {
bool prof_on();
// Records an event pair around the launches made between begin and end on
// stream s under `name`.  No-ops when profiling is off.
void prof_begin(const char *name, hipStream_t s);
void prof_end(const char *name, hipStream_t s);
}  // namespace schedk

#define SCHED_PROF_LAUNCH(name, stream, launch) \
  do {                                          \
    schedk::prof_begin(name, stream);           \
    launch;                                     \
    schedk::prof_end(name, stream);             \
  } while (0)

#define SCHED_PROF_LAUNCH_GRAPH(name, stream, call) \
  do {                                             \
    schedk::prof_begin(name, stream);              \
    {                                              \
      hipError_t _ge = (call);                     \
      if (_ge != hipSuccess) {                     \
        schedk::prof_end(name, stream);            \
        SCHED_HIP_TRY(_ge);                        \
      }                                            \
    }                                              \
    schedk::prof_end(name, stream);                \
  } while (0)
