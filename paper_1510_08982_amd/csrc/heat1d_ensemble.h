// heat1d_ensemble.h -- launcher of the ensemble kernel: many emulated
// asynchronous runs of equal rods, one workgroup per member.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heat1d {

struct EnsembleLaunch {
  int dtype;              // 0 FP32, 1 FP64
  const void* u0;         // E rods of N points, back to back
  void* uK;               // E rods of N points, or nullptr
  void* traj = nullptr;   // E x (K+1) states of N points (updated points written), or nullptr
  const uint64_t* seeds;  // E delay seeds (device)
  double* norms;          // E * (K/every + 1) doubles, or nullptr
  int64_t E;
  int32_t N, P, K, d, every;
  int32_t periodic;       // 1: ring of N points (c1, cN unused), 0: Dirichlet ends
  double r, c1, cN;
  // states at chosen steps: snaps + (e*nsnap + j)*N holds u(snap_steps[j]) of
  // member e (whole rod, ends included); snap_steps strictly increasing in [0, K]
  void* snaps = nullptr;
  int32_t nsnap = 0;
  int32_t snap_steps[64] = {};
};
constexpr int kEnsembleMaxSnaps = 64;

// LDS bytes one member needs: the last d+2 states of its rod, two rows of one
// delay byte per subdomain edge, and the per-wavefront norm partials.
int64_t ensemble_lds_bytes(int dtype, int64_t N, int64_t P, int d);
// Largest LDS footprint a member may have (one workgroup's static limit).
constexpr int64_t kEnsembleMaxLds = 65536;

hipError_t launch_ensemble(const EnsembleLaunch& a, hipStream_t s);

// Adjoint of the emulated asynchronous ensemble (Dirichlet ends or ring): one
// workgroup per member reverses its run from the trajectory the forward
// launch stored (EnsembleLaunch::traj).
struct EnsembleAdjointLaunch {
  int dtype;
  const void* traj;       // E x (K+1) states of N points
  const void* gK;         // E x N: dL/du(K)
  const uint64_t* seeds;  // E
  void* grad_u0;          // E x N (ends 0)
  double* grad_r;         // E
  double* grad_c1;        // E
  double* grad_cN;        // E
  int64_t E;
  int32_t N, P, K, d;
  int32_t periodic;       // 1: ring of N points (grad_c1, grad_cN written as 0)
  double r, c1, cN;
};
int64_t ensemble_adjoint_lds_bytes(int dtype, int64_t N, int64_t P, int d);
hipError_t launch_ensemble_adjoint(const EnsembleAdjointLaunch& a, hipStream_t s);

}  // namespace heat1d
