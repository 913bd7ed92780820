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

struct SolveItem {
  sfft_desc d;
  const double* G;
  const double* h;
  double* coef;
  sfft_solve_info* info;
  unsigned char* ws;
};

struct SolveBatch;
SolveBatch* solve_batch_create(const SolveItem* items, int n, int max_refine, int P, int num_cus,
                               hipError_t* err);
size_t solve_batch_dev_bytes(const SolveBatch* b);
hipError_t solve_batch_upload(SolveBatch* b, unsigned char* dev);
hipError_t solve_batch_launch(const SolveBatch* b, const Prof* pf, hipStream_t st);
int solve_batch_team(const SolveBatch* b);
void solve_batch_destroy(SolveBatch* b);

struct SubItem {
  sfft_desc d;
  const void* R;
  const void* S;
  const double* coef;
  void* D;
  double* chi2;
  unsigned char* ws;
};

struct SubBatch;
SubBatch* sub_batch_create(const SubItem* items, int n, int tile_rows, hipError_t* err);
size_t sub_batch_dev_bytes(const SubBatch* b);
hipError_t sub_batch_upload(SubBatch* b, unsigned char* dev);
hipError_t sub_batch_launch(const SubBatch* b, const Prof* pf, hipStream_t st);
void sub_batch_destroy(SubBatch* b);

}  // namespace sfft
