// Mini-batch k-means quantisation: the QUANTIZE step of Alg. 1 (Sec. 3.6),
// with the mini-batch algorithm of Sculley (2010) that the paper uses.
//
// Pixels are rows of m channels (FP32 in memory, FP64 arithmetic).  Per
// iteration t the batch M_t (pixel indices, drawn by the caller) is first
// assigned to the nearest centre under the centres at the start of the
// iteration; then, in batch order, each sample x with centre c = d[x] does
//   v[c] += 1,  eta = 1 / v[c],  c <- (1 - eta) c + eta x
// (v starts at 0, so a centre's first sample replaces it).  After the last
// iteration every pixel gets the index of its nearest centre (ties: the
// lowest index); pixels outside the mask get 0.
//
// The file is compiled with floating-point contraction off: every product
// and sum is rounded on its own, in the order written, so the centres and
// labels equal those of a plain FP64 evaluation of the same steps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace cmif {

constexpr int kKmMaxK = 64;
constexpr int kKmMaxM = 8;
constexpr int kKmMaxBatch = 8192;
constexpr int kKmThreads = 256;

// Squared distance of pixel x (m channels) to centre j, channels summed in
// order.
__device__ __forceinline__ double km_dist(const double* x, const double* cj,
                                          int m) {
  double d = 0.0;
  for (int ch = 0; ch < m; ++ch) {
    const double e = x[ch] - cj[ch];
    d = d + e * e;
  }
  return d;
}

__device__ __forceinline__ int km_nearest(const double* x, const double* c,
                                          int k, int m) {
  int best = 0;
  double bd = km_dist(x, c, m);
  for (int j = 1; j < k; ++j) {
    const double dj = km_dist(x, c + j * m, m);
    if (dj < bd) {
      bd = dj;
      best = j;
    }
  }
  return best;
}

// One workgroup runs every iteration: parallel assignment of the batch,
// then one thread per centre applies its samples in batch order.
// Indices outside [0, n) are skipped (they neither count nor move a centre;
// an initial centre from such an index is 0) and counted in *bad.
__global__ void __launch_bounds__(kKmThreads)
k_kmeans_fit(const float* __restrict__ img, int64_t n, int m, int k,
             const int32_t* __restrict__ init_idx,
             const int32_t* __restrict__ batches, int iters, int batch,
             double* __restrict__ centers, uint32_t* __restrict__ bad) {
  __shared__ double c[kKmMaxK * kKmMaxM];
  __shared__ int64_t v[kKmMaxK];
  __shared__ int8_t d[kKmMaxBatch];
  const int tid = threadIdx.x;
  // initial centres: the pixels init_idx (Sculley's random examples), or
  // the values already in `centers`
  for (int e = tid; e < k * m; e += blockDim.x) {
    double val = centers[e];
    if (init_idx != nullptr) {
      const int32_t idx = init_idx[e / m];
      val = 0.0;
      if (idx >= 0 && (int64_t)idx < n) val = (double)img[(int64_t)idx * m + e % m];
      else if (e % m == 0 && bad) atomicAdd(bad, 1u);
    }
    c[e] = val;
  }
  for (int j = tid; j < k; j += blockDim.x) v[j] = 0;
  __syncthreads();
  for (int t = 0; t < iters; ++t) {
    const int32_t* bt = batches + (int64_t)t * batch;
    for (int s = tid; s < batch; s += blockDim.x) {
      const int32_t idx = bt[s];
      int8_t lab = -1;
      if (idx >= 0 && (int64_t)idx < n) {
        double x[kKmMaxM];
        for (int ch = 0; ch < m; ++ch) x[ch] = (double)img[(int64_t)idx * m + ch];
        lab = (int8_t)km_nearest(x, c, k, m);
      } else if (bad) {
        atomicAdd(bad, 1u);
      }
      d[s] = lab;
    }
    __syncthreads();
    if (tid < k) {
      double cj[kKmMaxM];
      for (int ch = 0; ch < m; ++ch) cj[ch] = c[tid * m + ch];
      int64_t vj = v[tid];
      for (int s = 0; s < batch; ++s) {
        if (d[s] != tid) continue;
        const int64_t idx = bt[s];
        vj += 1;
        const double eta = 1.0 / (double)vj;
        const double keep = 1.0 - eta;
        for (int ch = 0; ch < m; ++ch)
          cj[ch] = keep * cj[ch] + eta * (double)img[idx * m + ch];
      }
      v[tid] = vj;
      for (int ch = 0; ch < m; ++ch) c[tid * m + ch] = cj[ch];
    }
    __syncthreads();
  }
  for (int e = tid; e < k * m; e += blockDim.x) centers[e] = c[e];
}

// Nearest-centre labels for every pixel (0 outside the mask).
__global__ void __launch_bounds__(kKmThreads)
k_kmeans_assign(const float* __restrict__ img, const uint8_t* __restrict__ mask,
                int64_t n, int m, int k, const double* __restrict__ centers,
                uint8_t* __restrict__ labels) {
  __shared__ double c[kKmMaxK * kKmMaxM];
  for (int e = threadIdx.x; e < k * m; e += blockDim.x) c[e] = centers[e];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    uint8_t lab = 0;
    if (mask == nullptr || mask[i] != 0) {
      double x[kKmMaxM];
      for (int ch = 0; ch < m; ++ch) x[ch] = (double)img[i * m + ch];
      lab = (uint8_t)km_nearest(x, c, k, m);
    }
    labels[i] = lab;
  }
}

hipError_t launch_kmeans(const KmeansArgs& a, hipStream_t st) {
  if (a.k < 1 || a.k > kKmMaxK || a.m < 1 || a.m > kKmMaxM || a.batch < 1 ||
      a.batch > kKmMaxBatch || a.iters < 0 || a.n < 1)
    return hipErrorInvalidValue;
  if (a.iters > 0 || a.init_idx != nullptr) {
    hipLaunchKernelGGL(k_kmeans_fit, dim3(1), dim3(kKmThreads), 0, st, a.img,
                       a.n, a.m, a.k, a.init_idx, a.batches, a.iters, a.batch,
                       a.centers, a.bad);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t want = (a.n + kKmThreads - 1) / kKmThreads;
  const int blocks = (int)(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(k_kmeans_assign, dim3(blocks), dim3(kKmThreads), 0, st,
                     a.img, a.mask, a.n, a.m, a.k, a.centers, a.labels);
  return hipGetLastError();
}

}  // namespace cmif
