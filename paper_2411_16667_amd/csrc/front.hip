// The result step on the device: the goal front P read out in lexicographic
// order (paper, Algorithm 1's return value; Section 3 defines the answer as
// a set, which is returned sorted so that two runs compare as sequences).
//
// P is an unordered array of d int32 planes with removed entries (INT32_MAX
// in every plane).  The live entries are listed first (tile counts, a scan,
// a scatter that keeps their order), then ordered by a stable least-significant
// -digit radix sort of the list: 8-bit digits, the last objective first and
// objective 0 last, only as many digits per objective as its largest live
// value needs.  Each sort pass is three launches: per-tile digit counts, one
// workgroup scanning the counts digit-major, and a stable scatter in which a
// lane's rank among same-digit lanes of its wave comes from eight ballots and
// the waves of a tile are ordered through LDS.  Output: the sorted cost rows
// (row-major, size x d) and the pool label id of each row.
#include "front.h"

namespace mos {

constexpr int FS_NT = 1024;              // threads (and items) per tile
constexpr int FS_WAVES = FS_NT / WAVE;
constexpr int FS_BINS = 256;

// live flag of entry i: a removed entry holds INT32_MAX in plane 0
__global__ __launch_bounds__(FS_NT) void k_fs_count_live(const int32_t* P0, int n,
                                                         int32_t* tile_cnt) {
  __shared__ int red[FS_WAVES];
  const int i = blockIdx.x * FS_NT + threadIdx.x;
  const bool live = i < n && P0[i] != INT32_MAX;
  const int c = __popcll(ballot(live));
  if (lane_id() == 0) red[threadIdx.x / WAVE] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < FS_WAVES; ++w) t += red[w];
    tile_cnt[blockIdx.x] = t;
  }
}

// Exclusive scan of cnt[0..m) in place by one workgroup (chunks of FS_NT with
// a running carry); *total receives the sum.
__global__ __launch_bounds__(FS_NT) void k_fs_scan(int32_t* cnt, int m, int32_t* total) {
  __shared__ int wsum[FS_WAVES];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < m; base += FS_NT) {
    const int i = base + threadIdx.x;
    const int v = i < m ? cnt[i] : 0;
    int x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane_id() >= o) x += y;
    }
    const int w = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) wsum[w] = x;
    __syncthreads();
    int before = carry;
    for (int u = 0; u < w; ++u) before += wsum[u];
    if (i < m) cnt[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == FS_NT - 1) carry = before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// Scatter the live entries' positions in their original order.
__global__ __launch_bounds__(FS_NT) void k_fs_list_live(const int32_t* P0, int n,
                                                        const int32_t* tile_off, int32_t* idx) {
  __shared__ int wcnt[FS_WAVES];
  const int i = blockIdx.x * FS_NT + threadIdx.x;
  const bool live = i < n && P0[i] != INT32_MAX;
  const uint64_t m = ballot(live);
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) wcnt[w] = __popcll(m);
  __syncthreads();
  int pos = tile_off[blockIdx.x];
  for (int u = 0; u < w; ++u) pos += wcnt[u];
  if (live) idx[pos + rank_below(m)] = i;
}

// Largest live value of every plane (for the number of digit passes).
__global__ __launch_bounds__(FS_NT) void k_fs_max(const int32_t* P, int64_t stride, int d,
                                                  const int32_t* idx, const int32_t* np,
                                                  int32_t* vmax) {
  const int n = *np;
  for (int k = blockIdx.y; k < d; k += gridDim.y) {
    int m = 0;
    for (int i = blockIdx.x * FS_NT + threadIdx.x; i < n; i += gridDim.x * FS_NT)
      m = max(m, P[(size_t)k * stride + idx[i]]);
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
    if (lane_id() == 0) atomicMax(&vmax[k], m);
  }
}

// Digit counts of one pass, digit-major: cnt[digit * ntiles + tile].
__global__ __launch_bounds__(FS_NT) void k_fs_digit_count(const int32_t* plane, const int32_t* idx,
                                                          const int32_t* np, int shift,
                                                          int32_t* cnt, int ntiles) {
  __shared__ int h[FS_BINS];
  const int n = *np;
  if (blockIdx.x * FS_NT >= n) {
    // tiles beyond the live count still own their (zero) counts
    if (threadIdx.x < FS_BINS) cnt[threadIdx.x * ntiles + blockIdx.x] = 0;
    return;
  }
  if (threadIdx.x < FS_BINS) h[threadIdx.x] = 0;
  __syncthreads();
  const int i = blockIdx.x * FS_NT + threadIdx.x;
  if (i < n) atomicAdd(&h[(plane[idx[i]] >> shift) & 255], 1);
  __syncthreads();
  if (threadIdx.x < FS_BINS) cnt[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one pass: out[pos] = in[i], pos = the scanned count of
// (digit, tile) + same-digit items before i in this tile.
__global__ __launch_bounds__(FS_NT) void k_fs_digit_scatter(const int32_t* plane,
                                                            const int32_t* in, const int32_t* np,
                                                            int shift, const int32_t* off,
                                                            int ntiles, int32_t* out) {
  __shared__ int wc[FS_WAVES][FS_BINS];
  const int n = *np;
  if (blockIdx.x * FS_NT >= n) return;
  const int w = threadIdx.x / WAVE;
  for (int x = threadIdx.x; x < FS_WAVES * FS_BINS; x += FS_NT) (&wc[0][0])[x] = 0;
  __syncthreads();
  const int i = blockIdx.x * FS_NT + threadIdx.x;
  const bool valid = i < n;
  const int item = valid ? in[i] : 0;
  const int dig = valid ? (plane[item] >> shift) & 255 : 0;
  // lanes of this wave holding the same digit
  uint64_t peers = ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t ones = ballot(valid && ((dig >> b) & 1));
    peers &= ((dig >> b) & 1) ? ones : ~ones;
  }
  const int r = rank_below(peers);
  if (valid && r == 0) wc[w][dig] = __popcll(peers);
  __syncthreads();
  if (valid) {
    int pos = off[dig * ntiles + blockIdx.x] + r;
    for (int u = 0; u < w; ++u) pos += wc[u][dig];
    out[pos] = item;
  }
}

// Rows of the sorted entries and their label ids.
__global__ void k_fs_gather(const int32_t* P, int64_t stride, const int32_t* lab, int d,
                            const int32_t* idx, const int32_t* np, int32_t* rows,
                            int32_t* labs) {
  const int n = *np;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int e = idx[i];
    for (int k = 0; k < d; ++k) rows[(size_t)i * d + k] = P[(size_t)k * stride + e];
    if (labs) labs[i] = lab[e];
  }
}

size_t front_sort_scratch_bytes(int n) {
  const int64_t nt = (n + FS_NT - 1) / FS_NT + 1;
  return (size_t)(2 * (int64_t)n + nt * FS_BINS + nt + 64) * 4 + 1024;
}

// Host part: the passes are chosen after reading the live count and the
// largest value of each plane back (two small copies).
int front_sort(const int32_t* P, int64_t stride, const int32_t* lab, int d, int n, void* scratch,
               int32_t* rows, int32_t* labs, hipStream_t st) {
  if (n <= 0) return 0;
  const int nt = (n + FS_NT - 1) / FS_NT;
  int32_t* w = (int32_t*)scratch;
  int32_t* idx_a = w;
  int32_t* idx_b = idx_a + n;
  int32_t* cnt = idx_b + n;                         // nt * FS_BINS (also the live tile counts)
  int32_t* small = cnt + (int64_t)(nt + 1) * FS_BINS;  // [0] live count, [1..d] plane maxima
  if (hipMemsetAsync(small, 0, 64 * 4, st) != hipSuccess) return -1;
  hipLaunchKernelGGL(k_fs_count_live, dim3(nt), dim3(FS_NT), 0, st, P, n, cnt);
  hipLaunchKernelGGL(k_fs_scan, dim3(1), dim3(FS_NT), 0, st, cnt, nt, small);
  hipLaunchKernelGGL(k_fs_list_live, dim3(nt), dim3(FS_NT), 0, st, P, n, cnt, idx_a);
  hipLaunchKernelGGL(k_fs_max, dim3(std::min(nt, 64), d), dim3(FS_NT), 0, st, P, stride, d,
                     idx_a, small, small + 1);
  int32_t hs[1 + MAXD];
  if (hipMemcpyAsync(hs, small, 4 * (1 + d), hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
  if (hipStreamSynchronize(st) != hipSuccess) return -1;
  const int np = hs[0];
  if (np == 0) return 0;
  const int ntl = (np + FS_NT - 1) / FS_NT;
  int32_t* cur = idx_a;
  int32_t* nxt = idx_b;
  for (int k = d - 1; k >= 0; --k) {
    int bits = 0;
    while (bits < 31 && (hs[1 + k] >> bits) != 0) ++bits;
    for (int shift = 0; shift < bits; shift += 8) {
      const int32_t* plane = P + (size_t)k * stride;
      hipLaunchKernelGGL(k_fs_digit_count, dim3(ntl), dim3(FS_NT), 0, st, plane, cur, small,
                         shift, cnt, ntl);
      hipLaunchKernelGGL(k_fs_scan, dim3(1), dim3(FS_NT), 0, st, cnt, ntl * FS_BINS,
                         (int32_t*)nullptr);
      hipLaunchKernelGGL(k_fs_digit_scatter, dim3(ntl), dim3(FS_NT), 0, st, plane, cur, small,
                         shift, cnt, ntl, nxt);
      std::swap(cur, nxt);
    }
  }
  const int gx = std::max(1, std::min(1024, (np + 255) / 256));
  hipLaunchKernelGGL(k_fs_gather, dim3(gx), dim3(256), 0, st, P, stride, lab, d, cur, small,
                     rows, labs);
  if (hipGetLastError() != hipSuccess) return -1;
  return np;
}

}  // namespace mos
