// Batched execution: per-phase launch interfaces shared by the build, solve
// and subtract translation units and the batch orchestration in the API.
#pragma once

#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace sfft {

// one pair of a batch
struct BuildItem {
  sfft_desc d;
  const void* R;
  const void* S;
  double* G;
  double* hv;
  unsigned char* ws;
};

struct BuildBatch;
BuildBatch* build_batch_create(const BuildItem* items, int n, const BuildPlan* plans, int rows_per_block,
                               hipError_t* err);
size_t build_batch_dev_bytes(const BuildBatch* b);
hipError_t build_batch_upload(BuildBatch* b, unsigned char* dev);
hipError_t build_batch_launch(const BuildBatch* b, const Prof* pf, hipStream_t st);
void build_batch_destroy(BuildBatch* b);

}  // namespace sfft
