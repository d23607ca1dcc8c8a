// Arguments of the on-device rebuild kernel (host and device side of the library).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "orchard_build.h"
#include "orchard_dev.h"

namespace orchard {

struct RebuildArgs {
  int32_t n_env;
  int64_t n_seg;
  build::DeriveConsts consts;
  // the descriptor as given at create (descriptor order)
  const int32_t* seg_off;     // [n_env + 1]
  const int32_t* parent;      // [n_seg] env-local
  const double* quat;         // [n_seg][4]
  const double* blen;         // [n_seg] length
  const double* rad;          // [n_seg]
  const double* rho;
  const double* E;
  const double* mor;
  const int32_t* apple_off;   // [n_env + 1]
  const int32_t* aseg;        // [n_apple] env-local segment
  const double* hang;         // [n_apple][3]
  const int32_t* int_of;      // descriptor segment -> internal node
  const int32_t* int_apple_of;  // descriptor apple -> internal apple
  const double* factors;      // [n_seg][4] length factor, radius factor, bend about x, about y (rad)
  double* work;               // 40 n_seg doubles
  int32_t* rejected;          // nullable: worlds left unchanged
  // the model's arrays (internal order)
  float4* rq;
  NodeRec* nrec;
  float4* geo;
  float* lenf;
  float* mmaxf;
  float* kp0;
  float* kd0;
  float* wmomf;
  float4* ahang;
  AppleRec* arec;
  float4* ahrest;
  double* ahrest64;           // [n_apple][3]
};

__global__ void k_rebuild(RebuildArgs A);

}  // namespace orchard
