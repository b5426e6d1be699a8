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
// Bracket `count` back-to-back launches of one kind with a single event pair
// (the operations inside do not record their own); the interval counts as
// `count` launches moving `bytes` in total, so the dispatch cost of the
// events is shared by the group.
void prof_group_begin(int kind, hipStream_t s, int count);
void prof_group_end(int kind, hipStream_t s, double bytes);

}  // namespace phs
