// Device-side recount of the hierarchy invariants (a checker, not part of the batch update).
//
// Every check is a single streaming pass with integer sums that are independent of the order of
// the additions (mod 2^64, or exact 128-bit), so the result is deterministic:
//   * row pass over one CSR orientation of one level: row sums against the stored degrees
//     (I6), positive weights, entries only between alive nodes, and weighted 64-bit
//     fingerprints sum_e w_e h(key_e) of the entries (two hash functions), of their transposed
//     keys, and of their keys mapped through the parents (the grouped sum of Eq. 3, I1), plus
//     the intra-community weight sum (Ein at level 0);
//   * node pass over one level: nested labels (I2), refined roots (I3), liveness of the level
//     above against the refined-community sizes, and at level 0 the community totals (I5):
//     fingerprints of sum_u kout(u) h(P(u)) against sum_c Kout(c) h(c), their plain sums and
//     the exact sum of Kout(c) Kin(c).
// Equal matrices give equal fingerprints; a matrix that differs in a single entry always gives a
// different one (h is odd and |w| < 2^63), and several differences cancel only by coincidence of
// the hash values.
#include "ldl_dev.h"
#include "ldl_check.h"

namespace ldl {

namespace {

constexpr int kTpb = 256;
constexpr unsigned kCheckBlocks = 1024;   // grid-stride loops: any n with a fixed grid

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}
// two independent odd hash values of a 64-bit key
__device__ __forceinline__ uint64_t h1(uint64_t k) { return mix64(k + 0x9e3779b97f4a7c15ull) | 1ull; }
__device__ __forceinline__ uint64_t h2(uint64_t k) { return mix64(k ^ 0xd1b54a32d192ed03ull) * 3ull + 1ull | 1ull; }
__device__ __forceinline__ uint64_t pk(uint32_t a, uint32_t b) { return ((uint64_t)a << 32) | b; }

__device__ __forceinline__ uint64_t wave_add_u64(uint64_t v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum kWords per-thread values over the block and add them to out[] with one atomic per word.
template <int kWords>
__device__ __forceinline__ void block_add(uint64_t (&v)[kWords], u64a* out) {
  __shared__ uint64_t part[kTpb / kWave][kWords];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < kWords; ++i) {
    const uint64_t s = wave_add_u64(v[i]);
    if (lane == 0) part[w][i] = s;
  }
  __syncthreads();
  if (threadIdx.x < kWords) {
    uint64_t s = 0;
    for (int j = 0; j < kTpb / kWave; ++j) s += part[j][threadIdx.x];
    if (s) atomicAdd(&out[threadIdx.x], (u64a)s);
  }
}

__device__ __forceinline__ int64_t wget(const CsrRef& c, uint64_t i) {
  return c.wide ? ((const int64_t*)c.w)[i] : (int64_t)((const uint32_t*)c.w)[i];
}

// One wavefront per row (grid stride).  transposed: the CSR holds in-rows (row = column of the
// matrix entry), so keys are (neighbour, row).
__global__ __launch_bounds__(kTpb) void k_inv_rows(CsrRef c, uint32_t n, const uint8_t* alive, const int64_t* deg,
                                                    const uint32_t* par, const uint32_t* lab, int transposed,
                                                    u64a* words, uint32_t* flags) {
  uint64_t acc[kInvRowWords];
#pragma unroll
  for (int i = 0; i < kInvRowWords; ++i) acc[i] = 0;
  uint32_t bad = 0;
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * blockDim.x / kWave;
  for (uint64_t u = wave; u < n; u += nwaves) {
    const uint32_t d = c.deg[u];
    const uint64_t o = c.off[u];
    const bool au = alive[u] != 0;
    const uint32_t pu = par ? par[u] : 0;
    const uint32_t lu = lab ? lab[u] : 0;
    int64_t rs = 0;
    for (uint32_t i = lane; i < d; i += kWave) {
      const uint32_t v = c.nbr[o + i];
      const int64_t w = wget(c, o + i);
      rs += w;
      if (v >= n) {
        bad |= kInvRange;
        continue;
      }
      if (w <= 0) bad |= kInvDegrees;
      if (!au || !alive[v]) bad |= kInvDegrees;
      const uint64_t key = transposed ? pk(v, (uint32_t)u) : pk((uint32_t)u, v);
      const uint64_t tkey = transposed ? pk((uint32_t)u, v) : pk(v, (uint32_t)u);
      const uint64_t uw = (uint64_t)w;
      acc[0] += 1;
      acc[1] += uw;
      acc[2] += uw * h1(key);
      acc[3] += uw * h2(key);
      acc[4] += uw * h1(tkey);
      acc[5] += uw * h2(tkey);
      if (par) {
        const uint32_t pv = par[v];
        const uint64_t akey = transposed ? pk(pv, pu) : pk(pu, pv);
        acc[6] += uw * h1(akey);
        acc[7] += uw * h2(akey);
      }
      if (lab && lab[v] == lu) acc[8] += uw;
    }
    rs = (int64_t)wave_add_u64((uint64_t)rs);
    if (lane == 0 && rs != deg[u]) bad |= kInvDegrees;
  }
  if (bad) atomicOr(flags, bad);
  block_add<kInvRowWords>(acc, words);
}

// One thread per node (grid stride) of level r.
//   up_* : level r+1 (null at the top level); K*: community totals (level 0 only)
__global__ __launch_bounds__(kTpb) void k_inv_nodes(uint32_t n, const uint8_t* alive, const uint32_t* lab,
                                                     const uint32_t* par, const uint32_t* rsize, const int64_t* kout,
                                                     const int64_t* kin, const uint8_t* up_alive,
                                                     const uint32_t* up_lab, const int64_t* Kout, const int64_t* Kin,
                                                     u64a* words, i64a* skk_hi, uint32_t* flags) {
  uint64_t acc[kInvNodeWords];
#pragma unroll
  for (int i = 0; i < kInvNodeWords; ++i) acc[i] = 0;
  i128 skk = 0;
  uint32_t bad = 0;
  for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (uint64_t)gridDim.x * blockDim.x) {
    const bool a = alive[u] != 0;
    if (!a && (kout[u] != 0 || kin[u] != 0)) bad |= kInvDegrees;
    if (up_alive) {
      // liveness of the level above follows the refined-community sizes; roots and nesting
      const bool au = up_alive[u] != 0;
      if (au != (rsize[u] > 0)) bad |= kInvAggregate;
      if (au && !(a && par[u] == u)) bad |= kInvRoots;
      if (a) {
        const uint32_t p = par[u];
        if (p >= n || !up_alive[p]) bad |= kInvAggregate;
        else if (up_lab[p] != lab[u]) bad |= kInvLabels;
        acc[0] += h1(p);
      }
      acc[1] += (uint64_t)rsize[u] * h1(u);
    }
    if (Kout) {
      const uint32_t l = lab[u];
      if (l >= n) {
        bad |= kInvRange;
      } else {
        acc[2] += (uint64_t)kout[u] * h1(l);
        acc[3] += (uint64_t)kin[u] * h2(l);
      }
      acc[4] += (uint64_t)Kout[u] * h1((uint64_t)u);
      acc[5] += (uint64_t)Kin[u] * h2((uint64_t)u);
      acc[6] += (uint64_t)Kout[u];
      acc[7] += (uint64_t)Kin[u];
      skk += (i128)Kout[u] * (i128)Kin[u];
    }
  }
  if (bad) atomicOr(flags, bad);
  if (Kout) {   // exact 128-bit block sum of Kout Kin, one atomic pair per block
    __shared__ uint64_t slo[kTpb / kWave];
    __shared__ int64_t shi[kTpb / kWave];
    for (int o = kWave / 2; o > 0; o >>= 1) {
      const uint64_t lo = __shfl_xor((uint64_t)skk, o, kWave);
      const int64_t hi = __shfl_xor((int64_t)(skk >> 64), o, kWave);
      skk += ((i128)hi << 64) | (i128)lo;
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) {
      slo[w] = (uint64_t)skk;
      shi[w] = (int64_t)(skk >> 64);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      i128 t = 0;
      for (int j = 0; j < kTpb / kWave; ++j) t += ((i128)shi[j] << 64) | (i128)slo[j];
      if (t != 0) atomic_add_i128(&words[kInvNodeWords], skk_hi, t);
    }
  }
  block_add<kInvNodeWords>(acc, words);
}

__global__ void k_inv_clear(u64a* words, uint32_t nwords) {
  for (uint32_t i = threadIdx.x; i < nwords; i += blockDim.x) words[i] = 0;
}

inline unsigned check_grid(uint64_t items, uint64_t per_block) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > kCheckBlocks) g = kCheckBlocks;
  return (unsigned)g;
}

}  // namespace

void launch_inv_clear(InvScratch* sc, hipStream_t s) {
  k_inv_clear<<<1, kTpb, 0, s>>>((u64a*)sc, (uint32_t)(sizeof(InvScratch) / 8));
}

void launch_inv_rows(CsrRef c, uint32_t n, const uint8_t* alive, const int64_t* deg, const uint32_t* par,
                     const uint32_t* lab, int transposed, InvScratch* sc, hipStream_t s) {
  if (n == 0 || !c.off) return;
  k_inv_rows<<<check_grid(n, kTpb / kWave), kTpb, 0, s>>>(c, n, alive, deg, par, lab, transposed,
                                                           transposed ? sc->in : sc->out, &sc->flags);
}

void launch_inv_nodes(uint32_t n, const uint8_t* alive, const uint32_t* lab, const uint32_t* par,
                      const uint32_t* rsize, const int64_t* kout, const int64_t* kin, const uint8_t* up_alive,
                      const uint32_t* up_lab, const int64_t* Kout, const int64_t* Kin, InvScratch* sc, hipStream_t s) {
  if (n == 0) return;
  k_inv_nodes<<<check_grid(n, kTpb), kTpb, 0, s>>>(n, alive, lab, par, rsize, kout, kin, up_alive, up_lab, Kout, Kin,
                                                    sc->node, (i64a*)&sc->skk_hi, &sc->flags);
}

}  // namespace ldl
