// Persistent batched solve (fe_batch.hip): device structures and launcher,
// driven by fe_solve_batched (fe_api.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "fe_kernels.h"

namespace fe {

// Lengths (each of nx, ny, nz) the persistent kernel is compiled for.
inline bool batch_length_ok(int n) {
  return n == 16 || n == 24 || n == 32 || n == 48 || n == 64 || n == 96 || n == 128;
}

constexpr int kBatchClasses = 8;  // grid classes of one persistent launch
constexpr int kBatchRunning = 100;  // sample state: still iterating

// One grid class of a batch: packed per-sample buffers and the workgroups of
// each pass per sample.
struct BatchClassDev {
  Dims d;
  float* eps[2];  // packed [sample][6][N], the iterate of parity 0 / 1
  float* R[2];    // packed [sample][3][N] (divergence, then displacement)
  cpx<float>* S;  // packed [sample][3][Hp ny nx]
  const uint8_t* phase;
  double* partials;  // [sample][bu][7]
  const PhaseCoef<float>* coef;
  int ncoef;
  const GreenConst<float>* gcon;
  const cpx<float>* tw[3];
  WaveTables<float> wt;
  int bz, by, bx, bu;  // workgroups per sample: z passes, y passes, x pass, divergence / update
  int zchunk;          // z planes per divergence / update workgroup
  int* act;            // active sample indices (within the class)
  int nact;
  int first;  // index of the class's sample 0 in the state array
  int n;
};

// Per-sample state, updated on the device after every iteration.
struct BatchState {
  int status;      // kBatchRunning, then the fe_status of the sample
  int iterations;  // iterations done
  int parity;      // buffer holding the current iterate
  int rising, best_k, pad;
  double eta, prev, best;
  double mean[6];
};

struct BatchDev {
  int ncls;
  BatchClassDev cls[kBatchClasses];
  BatchState* st;
  double tol;
  int max_iter, diverge_window;
  int* ctrl;  // ctrl[0]: active samples after the last compaction; ctrl[1]: a barrier timed out
  unsigned long long* bar;  // grid barrier counter, zero at the launch
};

// Workgroups per sample of each pass and the update's z chunk for a grid
// whose lengths satisfy batch_length_ok.
void batch_class_layout(const Dims& d, int* bz, int* by, int* bx, int* bu, int* zchunk);

// Resident workgroups of the persistent kernel on the current device (the
// grid of a cooperative launch), 0 if cooperative launches are unavailable.
int batch_persistent_grid(int op, bool accel);

// One cooperative launch over the batch described by dev (device memory).
hipError_t launch_batch_persistent(int op, bool accel, BatchDev* dev, int grid, hipStream_t s);

}  // namespace fe
