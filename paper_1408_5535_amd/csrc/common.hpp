// Shared helpers of the PHSVDS HIP library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace phs {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define PHS_HIP(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::phs::Error(-3, std::string(#call) + ": " + hipGetErrorString(e_));       \
  } while (0)

#define PHS_CHECK_LAUNCH() PHS_HIP(hipGetLastError())

#define PHS_REQUIRE(cond, code, msg)                                                     \
  do {                                                                                   \
    if (!(cond)) throw ::phs::Error((code), (msg));                                      \
  } while (0)

constexpr int kEinval = -1;
constexpr int kEbreak = -2;
constexpr int kEnomem = -4;

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// SplitMix64 (Steele, Lea & Flood 2014): output for state x is mix(x + gamma).
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Entry j of random stream s for seed t, uniform in [-0.5, 0.5).
__host__ __device__ inline double stream_uniform(uint64_t seed, uint64_t s, uint64_t j) {
  uint64_t key = (seed << 40) + (s << 24) + j;
  return (double)(splitmix64(key) >> 11) * 0x1.0p-53 - 0.5;
}

// Bump allocator over a caller-provided device workspace.
struct Arena {
  char *base = nullptr;
  size_t size = 0, used = 0;
  bool dry = false;  // size-only planning pass
  template <typename T>
  T *take(int64_t count) {
    size_t bytes = ((size_t)count * sizeof(T) + 255) & ~(size_t)255;
    size_t at = used;
    used += bytes;
    if (dry) return nullptr;
    if (used > size) throw Error(kEnomem, "workspace too small");
    return reinterpret_cast<T *>(base + at);
  }
};

}  // namespace phs
