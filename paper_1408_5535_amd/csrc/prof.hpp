// Optional per-kernel timing with HIP events on the launching stream.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace phs {

enum ProfKind { kProfSpmm64 = 0, kProfSpmm32, kProfTn, kProfNn, kProfRitz, kProfCount };

bool prof_on();
// Bracket one logical operation; `bytes` is its algorithmic HBM traffic.
void prof_begin(int kind, hipStream_t s);
void prof_end(int kind, hipStream_t s, double bytes);

}  // namespace phs
