// qmc_jit.h -- run-time specialisation of the evaluation kernel to one integrand.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "qmc_device.h"

namespace qmcj {

// What the generated code depends on (coefficients are read from memory).
struct Spec {
  uint32_t dim, n_u, n_f;
  const uint8_t* expo;  // [(n_u + n_f) * dim]
  int pu_mode, pu_k, pf_mode, pf_k;
  int tk;  // qmcd::TK_*
  int S;   // shifts per thread group
  int vr;  // variance-reduction map compiled in (1) or out (0)
  int cplx = 0;  // deformed (complex) integrand
  // > 0: real f = prefactor (U^ru F^rf)^(-1/2), one reciprocal square root for
  // both powers (pow_u = -ru/2, pow_f = -rf/2); 0: the separate powers
  int ru = 0, rf = 0;
  // complex integrands: coefficient values [n_u + n_f] and, with vr, the map
  // parameters [dim][6] compiled into the kernel as constants (nullptr: read
  // from the kernel's arguments)
  const double* coef = nullptr;
  const double* vr_params = nullptr;
};

struct Kernel {
  hipFunction_t f32 = nullptr, f64 = nullptr;  // 32-bit / 64-bit index stepping
  int occ_blocks = 0;                           // resident blocks per CU
  // real integrands: persistent batch kernel over a tile list (the
  // arguments of the table-driven batch kernels), S_REAL shifts per group
  hipFunction_t batch = nullptr;
  int occ_batch = 0;
};

std::string generate(const Spec& s);
// Compile (or fetch from the cache) the specialised kernels for the current device.
int get(int device, const Spec& s, Kernel* out);
// Generate and compile only (no device needed); code size in bytes.
int compile_only(const Spec& s, size_t* code_bytes);
hipError_t launch(const Kernel& k, bool idx32, const qmcd::EvalArgs& a, dim3 grid, hipStream_t st);
hipError_t launch_batch(const Kernel& k, const qmcd::EvalArgs* items, const uint32_t* order, const uint32_t* prefix,
                        uint32_t nitems, uint32_t* counter, uint32_t blocks, hipStream_t st);
const char* last_error();

}  // namespace qmcj
