// Counting sort of the particle arrays by element (active particles first,
// in element order; inactive ones at the end).  Histogram with atomics, an
// exclusive scan over the E+1 buckets, then a scatter of every SoA field.
#include "fp_launch.h"

namespace fp {

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// rank of each particle within its bucket.  The particles are mostly in
// element order already (sorted at the last step, few crossings since), so
// neighbouring lanes share keys: one atomic per run of equal keys within a
// wavefront instead of one per particle (atomics on one address serialise)
__global__ __launch_bounds__(256) void k_sort_hist(const int8_t* __restrict__ status,
                                                   const int32_t* __restrict__ elem, int64_t n, int E,
                                                   int32_t* count, int32_t* rank) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool valid = p < n;
  const int key = valid ? (status[p] == ACTIVE ? elem[p] : E) : -1;
  const int prev = __shfl_up(key, 1, 64);
  const bool head = valid && (lane == 0 || prev != key);
  const unsigned long long heads = __ballot(head);
  const int nvalid = (int)__popcll(__ballot(valid));   // the valid lanes are a prefix
  int base = 0;
  if (head) {
    const unsigned long long above = lane == 63 ? 0ull : heads >> (lane + 1);
    const int next = above ? lane + 1 + __builtin_ctzll(above) : nvalid;
    base = atomicAdd(count + key, next - lane);
  }
  // the head of this lane's run: the highest head at or below the lane
  const unsigned long long upto = heads & (lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull));
  const int start = upto ? 63 - __builtin_clzll(upto) : 0;
  const int b = __shfl(base, start, 64);
  if (valid) rank[p] = b + (lane - start);
}

// exclusive scan of 1024-entry tiles (256 threads x 4), tile totals to sums
__global__ __launch_bounds__(256) void k_scan_tiles(const int32_t* in, int32_t* out, int64_t n, int32_t* sums) {
  __shared__ int32_t sh[256];
  int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
  int32_t v[4], s = 0;
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    s += v[k];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int32_t t = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = sh[threadIdx.x] - s;
  for (int k = 0; k < 4; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 255) sums[blockIdx.x] = sh[255];
}

// exclusive scan of the tile totals by one block (loops over chunks of 1024)
__global__ __launch_bounds__(256) void k_scan_sums(int32_t* sums, int64_t nt) {
  __shared__ int32_t sh[256];
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < nt; c0 += 1024) {
    int64_t base = c0 + threadIdx.x * 4;
    int32_t v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
      v[k] = (base + k < nt) ? sums[base + k] : 0;
      s += v[k];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      int32_t t = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    int32_t run = carry + sh[threadIdx.x] - s;
    for (int k = 0; k < 4; ++k) {
      if (base + k < nt) sums[base + k] = run;
      run += v[k];
    }
    int32_t tot = sh[255];
    __syncthreads();
    carry += tot;
  }
}

__global__ void k_scan_add(int32_t* out, int64_t n, const int32_t* sums) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / 1024];
}

__global__ __launch_bounds__(256) void k_sort_scatter(Particles S, Particles D, int64_t n, int E,
                                                      const int32_t* __restrict__ start,
                                                      const int32_t* __restrict__ rank) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int8_t st = S.status[p];
  int32_t e = S.elem[p];
  int key = st == ACTIVE ? e : E;
  int64_t q = (int64_t)start[key] + rank[p];
  const int64_t cs = S.cap, cd = D.cap;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    D.x[k * cd + q] = S.x[k * cs + p];
    D.v[k * cd + q] = S.v[k * cs + p];
    D.kx[k * cd + q] = S.kx[k * cs + p];
    D.kv[k * cd + q] = S.kv[k * cs + p];
    D.xi[k * cd + q] = S.xi[k * cs + p];
  }
  D.d[q] = S.d[p];
  D.elem[q] = e;
  D.hits[q] = S.hits[p];
  D.id[q] = S.id[p];
  D.status[q] = st;
}

hipError_t scan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* sums, hipStream_t s) {
  int64_t nt = (n + 1023) / 1024;
  k_scan_tiles<<<dim3((unsigned)nt), 256, 0, s>>>(in, out, n, sums);
  k_scan_sums<<<1, 256, 0, s>>>(sums, nt);
  k_scan_add<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(out, n, sums);
  return hipGetLastError();
}

hipError_t launch_sort(const Particles& src, const Particles& dst, int64_t n, int E, int32_t* count, int32_t* start,
                       int32_t* rank, int32_t* block_sums, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t nb = E + 1;
  k_fill_i32<<<dim3((unsigned)((nb + 255) / 256)), 256, 0, s>>>(count, nb, 0);
  k_sort_hist<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(src.status, src.elem, n, E, count, rank);
  hipError_t err = scan_i32(count, start, nb, block_sums, s);
  if (err != hipSuccess) return err;
  k_sort_scatter<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(src, dst, n, E, start, rank);
  return hipGetLastError();
}

}  // namespace fp
