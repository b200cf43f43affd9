// Optional per-kernel timing with HIP events (off unless dect_profile_start was called).
#pragma once

#include "common.h"

namespace dect {

bool prof_enabled();
int prof_begin(const char* name, hipStream_t s);
void prof_end(int token, hipStream_t s);

// Times the launches made in its scope when profiling is on.
struct ProfScope {
    int token;
    hipStream_t s;
    ProfScope(const char* name, hipStream_t st) : token(prof_begin(name, st)), s(st) {}
    ~ProfScope() { prof_end(token, s); }
};

}  // namespace dect
