// Persistent-kernel instantiations: one translation unit per workgroup width
// (built with SBT_TPE set), each holding one kernel per LDS slot capacity.
#pragma once

namespace sbt {

// LDS slot capacities with a compiled persistent kernel (0: every event reads
// its modules from memory); a requested capacity is rounded down to one.
constexpr int kCaps[] = {0, 256, 448, 672, 768, 1024, 1536};
constexpr int kNumCaps = 7;

// host stub of the persistent kernel of width tpe for an instantiated
// capacity, or nullptr
const void *persistent_kernel_64(int cap);
const void *persistent_kernel_128(int cap);
const void *persistent_kernel_256(int cap);
const void *persistent_kernel_512(int cap);
const void *persistent_kernel_1024(int cap);
// the 512-lane kernel held to six waves per SIMD, for three workgroups per
// compute unit; compiled for 448-hit slots only (nullptr otherwise)
const void *persistent_kernel_512_dense(int cap);

}  // namespace sbt
