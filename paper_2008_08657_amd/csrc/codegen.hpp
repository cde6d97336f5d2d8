// Scan kernels generated per group and compiled at prepare time (hipRTC).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "engine.hpp"

namespace lmfao {

struct GenKernel {
  hipFunction_t fn = nullptr;
  std::vector<uint64_t> args;   // argument words the kernel reads (pointers and counts)
  int lds = 0;                  // dynamic LDS bytes
  int block = 0;                // threads per workgroup
  std::string source;
};

// Generates and compiles the scan of a lean scan descriptor.  Returns false
// with a reason when the descriptor is outside what the generator handles or
// compilation fails; the caller then launches the generic lean kernel.
bool gen_scan_kernel(const DScan& d, int n_atoms, bool f64, const std::string& tag, GenKernel& out,
                     std::string& why);

// hipRTC compile of `src` for gfx950 and load of the function `name`.
bool compile_kernel(const std::string& src, const char* name, hipFunction_t& fn, std::string& why);

}  // namespace lmfao
