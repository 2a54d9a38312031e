// Status checks of HIP runtime calls and kernel launches (device sources).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "common.hpp"

#define HIPCHECK(expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      ::kifmm::raise(KIFMM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

#define LAUNCHCHECK(what)                                                                \
  do {                                                                                   \
    hipError_t e_ = hipGetLastError();                                                   \
    if (e_ != hipSuccess)                                                                \
      ::kifmm::raise(KIFMM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e_));   \
  } while (0)
