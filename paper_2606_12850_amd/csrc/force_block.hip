// FP32 element internal-force kernel on 2 x 2 x 2 element blocks (NGLL <= 5).
//
// The operator is that of force_f32.hip (Sec. II-B weak form: gather, three
// forward contractions with D, inverse-Jacobian map, isotropic stress,
// weighted transpose contractions, assembly; Sec. IV-D fused traversal), but
// one workgroup owns eight face-adjacent elements that form a cube of
// (2n - 1)^3 nodes (729 at NGLL 5), and the colouring is over blocks: the
// block launches of one colour touch disjoint node sets (Sec. IV-C colouring,
// one level up).  In the per-element kernel a parity colour spreads over the
// whole domain, so every launch gathers and read-modify-writes partial
// 128-byte lines of u and f and each node's lines are fetched by several
// launches.  Here each node of a block is gathered once and stored once, as
// rows of 2n - 1 consecutive nodes:
//   * node lanes (lane < (2n-1)^3): u of the block's nodes into LDS, and at
//     the end the block's nodal force (prior f, zero at first-touch nodes,
//     plus the summed element contributions) back to f;
//   * element lanes (lane = 128 m + p, p < n^3): element m = dx + 2 dy + 4 dz
//     of the block at its point p, reading u from the block's node array,
//     writing its force contribution to LDS; the nodal sum takes the up to
//     eight contributions of a node in a fixed order (deterministic).
// Elements must be affine-numbered with the block's strides; the host builds
// the blocks and falls back to the per-element kernel when a mesh does not
// decompose into them.
#include "elem_common.hpp"

namespace semx {
namespace {

constexpr int kBlockLanes = 1024;

template <int NG>
struct BlockShape {
  static constexpr int N3 = NG * NG * NG;
  static constexpr int ND = NG * NG;
  static constexpr int NB1 = 2 * NG - 1;            // nodes along a block edge
  static constexpr int NBN = NB1 * NB1 * NB1;        // nodes of a block
  static constexpr int NWB = (NBN + 31) / 32;        // first-touch words per block
  static_assert(8 * 128 == kBlockLanes && N3 <= 128, "eight elements of at most 128 points");
  static_assert(NBN <= kBlockLanes, "one node per lane");
};

// The block's node span: raw buffer resources over its nodes in u and f and
// the lane's byte offset (node lanes); out of range for the other lanes,
// which then read zeros and fetch nothing.
struct BlockSpan {
  __amdgpu_buffer_rsrc_t ru, rf;
  int off;
};

template <int NG>
__device__ __forceinline__ BlockSpan block_span(const ForceArgs& a, const BlockArgs& b, int blk, const float* u,
                                                float* f, int lane) {
  using S = BlockShape<NG>;
  const int* r = b.baff + (size_t)blk * 4;
  const int sx = r[1], sy = r[2], sz = r[3];
  const int lo = (S::NB1 - 1) * (min(sx, 0) + min(sy, 0) + min(sz, 0));
  const int gmin = r[0] + lo;
  const int bytes = ((S::NB1 - 1) * (abs(sx) + abs(sy) + abs(sz)) + 1) * 12;
  BlockSpan s;
  s.ru = __builtin_amdgcn_make_buffer_rsrc((void*)(u + 3 * (size_t)gmin), (short)0, bytes, kBufferWord3);
  s.rf = __builtin_amdgcn_make_buffer_rsrc((void*)(f + 3 * (size_t)gmin), (short)0, bytes, kBufferWord3);
  const int X = lane % S::NB1, Y = (lane / S::NB1) % S::NB1, Z = lane / (S::NB1 * S::NB1);
  s.off = lane < S::NBN ? (X * sx + Y * sy + Z * sz - lo) * 12 : INT32_MIN;
  return s;
}

// First-touch bit of the lane's node: bit n & 31 of word n >> 5 of the
// block's words; wave w holds nodes 64 w .. 64 w + 63 (words 2w, 2w + 1).
template <int NG>
__device__ __forceinline__ bool block_first(const BlockArgs& b, int blk) {
  using S = BlockShape<NG>;
  if (!b.bfirst) return false;
  const uint32_t* w = b.bfirst + (size_t)blk * S::NWB;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const uint64_t lo = wave * 2 < S::NWB ? w[wave * 2] : 0u;
  const uint64_t hi = wave * 2 + 1 < S::NWB ? w[wave * 2 + 1] : 0u;
  return __builtin_amdgcn_inverse_ballot_w64(lo | (hi << 32));
}

// Forward contractions of element m at point (i, j, k), reading u from the
// block's node array (stride 1, NB1, NB1^2 along xi, eta, zeta).
template <int NG>
__device__ __forceinline__ void block_grad(const float* s_un, const float* s_D, int base, int i, int j, int k,
                                           float du[3][3]) {
  using S = BlockShape<NG>;
  constexpr int NB1 = S::NB1, NBN = S::NBN;
#pragma unroll
  for (int c = 0; c < 3; ++c) du[c][0] = du[c][1] = du[c][2] = 0.0f;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const float di = s_D[i * NG + q], dj = s_D[j * NG + q], dk = s_D[k * NG + q];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      du[c][0] += di * s_un[c * NBN + base + q + NB1 * (j + NB1 * k)];
      du[c][1] += dj * s_un[c * NBN + base + i + NB1 * (q + NB1 * k)];
      du[c][2] += dk * s_un[c * NBN + base + i + NB1 * (j + NB1 * q)];
    }
  }
}

// One workgroup per block (SKEL: the memory skeleton, the same loads and
// stores without the arithmetic).  Node coordinate X of the block and point
// ix of element dx along xi are related by X = (NG - 1) dx + ix.
template <int NG, int GEO, bool SKEL>
__global__ __launch_bounds__(kBlockLanes) void force_block_kernel(ForceArgs a, BlockArgs b) {
  using S = BlockShape<NG>;
  constexpr int N3 = S::N3, ND = S::ND, NB1 = S::NB1, NBN = S::NBN;
  __shared__ float s_un[3 * NBN];       // u at the block's nodes (component-major)
  __shared__ float s_fp[3 * NBN];       // prior force at the block's nodes
  __shared__ float s_q[8 * 9 * N3];     // weighted fluxes, per element
  __shared__ float s_F[8 * 3 * N3];     // element-point forces, per element
  __shared__ float s_D[ND + NG];        // D (row-major), then the GLL nodes

  const int nblk = (int)b.count;
  const int bi = xcd_group(nblk);
  if (bi >= nblk) return;  // uniform over the block
  const int blk = (int)b.beg + bi;

  const int lane = threadIdx.x;
  const int m = __builtin_amdgcn_readfirstlane(lane >> 7);  // element of the block: waves 2m, 2m + 1
  const int p = lane & 127;
  const bool act = p < N3;
  const int pp = act ? p : 0;
  const int i = pp % NG, j = (pp / NG) % NG, k = pp / ND;
  const int base = (NG - 1) * ((m & 1) + NB1 * (((m >> 1) & 1) + NB1 * (m >> 2)));

  const int model = blockIdx.y;
  const float* __restrict__ u = a.u + (size_t)model * a.nglob * 3;
  float* f = a.f + (size_t)model * a.nglob * 3;
  const float* __restrict__ mat = a.mat + (size_t)model * a.nspec * 2 * N3;
  const int pos = b.bpos[(size_t)blk * 8 + m];  // launch position of element m (uniform over the wave)

  float tab = 0.0f;
  if (lane < ND) tab = a.D[lane];
  else if (GEO == kTrilinear && lane < ND + NG) tab = a.xi[lane - ND];
  ElemGeom<GEO> eg;
  load_elem_geom<GEO>(a, pos, eg);
  float G[9];
  if constexpr (GEO == kStored) {
    const float* gp = a.gam_pt + (size_t)pos * 9 * N3 + pp;
#pragma unroll
    for (int d = 0; d < 9; ++d) G[d] = ldnt(gp + d * N3);
  }
  const float lw = ldnt(mat + (size_t)pos * 2 * N3 + pp);
  const float mw = ldnt(mat + (size_t)pos * 2 * N3 + N3 + pp);
  const BlockSpan sp = block_span<NG>(a, b, blk, u, f, lane);
  float uo[3], fo[3];
  buf_load<3>(sp.ru, sp.off, uo);
  // prior force at the lane's node (zero at first-touch nodes, nothing
  // fetched there), requested with u: both arrive by the first barrier and
  // wait in LDS for the nodal sum, so no register holds them meanwhile
  buf_load<3>(sp.rf, block_first<NG>(b, blk) ? INT32_MIN : sp.off, fo);
  pin_elem_geom<GEO>(eg);
  if (lane < ND + NG) s_D[lane] = tab;
  if (lane < NBN) {
    s_un[lane] = uo[0];
    s_un[NBN + lane] = uo[1];
    s_un[2 * NBN + lane] = uo[2];
    s_fp[lane] = fo[0];
    s_fp[NBN + lane] = fo[1];
    s_fp[2 * NBN + lane] = fo[2];
  }
  __syncthreads();

  if constexpr (SKEL) {
    // memory skeleton: the same loads and stores, no arithmetic
    float s = lw + mw;
    if constexpr (GEO == kStored) {
#pragma unroll
      for (int d = 0; d < 9; ++d) s += G[d];
    } else {
#pragma unroll
      for (int d = 0; d < ElemGeom<GEO>::NS; ++d) s += eg.v[d];
    }
    if (act) s_F[m * 3 * N3 + pp] = s;
    __syncthreads();
    __syncthreads();
    if (lane < NBN) {
      const float out[3] = {s_fp[lane] + s_F[lane] * s_un[lane], s_fp[NBN + lane] + s_un[NBN + lane],
                            s_fp[2 * NBN + lane] + s_un[2 * NBN + lane]};
      semx_v3u v;
      v.x = __float_as_uint(out[0]);
      v.y = __float_as_uint(out[1]);
      v.z = __float_as_uint(out[2]);
      __builtin_amdgcn_raw_buffer_store_b96(v, sp.rf, sp.off, 0, 0);
    }
    return;
  }

  float rx = 0.f, ry = 0.f, rz = 0.f;  // reference coordinates (trilinear path)
  if constexpr (GEO == kTrilinear) {
    rx = s_D[ND + i];
    ry = s_D[ND + j];
    rz = s_D[ND + k];
  }
  float du[3][3];
  block_grad<NG>(s_un, s_D, base, i, j, k, du);
  float Mg[9], scale, det;
  geom_map_from<GEO>(eg.v, G, rx, ry, rz, Mg, scale, det);
  float gr[3][3];
  apply_map(du, Mg, gr);
  stress_flux(gr, lw, mw, scale, Mg, s_q + m * 9 * N3, N3, pp, act);
  __syncthreads();

  float F[3];
  ref_div<NG>(s_q + m * 9 * N3, s_D, i, j, k, F);
  if (act) {
    s_F[m * 3 * N3 + pp] = F[0];
    s_F[m * 3 * N3 + N3 + pp] = F[1];
    s_F[m * 3 * N3 + 2 * N3 + pp] = F[2];
  }
  __syncthreads();

  if (lane < NBN) {
    // the node's contributions: along each axis the primary element (the one
    // whose interior or lower face holds the coordinate) and, on the block's
    // middle plane, the upper element at its point 0; the index of element
    // (ex, ey, ez) at point (ix, jy, kz) in s_F is a sum of one term per axis
    const int X = lane % NB1, Y = (lane / NB1) % NB1, Z = lane / (NB1 * NB1);
    const int px = X >= NG ? 1 : 0, py = Y >= NG ? 1 : 0, pz = Z >= NG ? 1 : 0;
    const int tx[2] = {px * 3 * N3 + (X - (NG - 1) * px), 3 * N3};
    const int ty[2] = {py * 6 * N3 + NG * (Y - (NG - 1) * py), 6 * N3};
    const int tz[2] = {pz * 12 * N3 + NG * NG * (Z - (NG - 1) * pz), 12 * N3};
    const bool hx = X == NG - 1, hy = Y == NG - 1, hz = Z == NG - 1;
    float acc[3] = {s_fp[lane], s_fp[NBN + lane], s_fp[2 * NBN + lane]};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int sxb = t & 1, syb = (t >> 1) & 1, szb = t >> 2;
      const bool use = (!sxb || hx) && (!syb || hy) && (!szb || hz);
      const int src = tx[sxb] + ty[syb] + tz[szb];
      if (use) {
        acc[0] += s_F[src];
        acc[1] += s_F[src + N3];
        acc[2] += s_F[src + 2 * N3];
      }
    }
    semx_v3u v;
    v.x = __float_as_uint(acc[0]);
    v.y = __float_as_uint(acc[1]);
    v.z = __float_as_uint(acc[2]);
    __builtin_amdgcn_raw_buffer_store_b96(v, sp.rf, sp.off, 0, 0);
  }
}

template <int NG, bool SKEL>
hipError_t launch_block_n(int geo, const ForceArgs& a, const BlockArgs& b, hipStream_t s) {
  if (b.count <= 0) return hipSuccess;
  const int64_t nb = ((b.count + kNumXcd - 1) / kNumXcd) * kNumXcd;
  dim3 grid((unsigned)nb, (unsigned)a.nmodels), block(kBlockLanes);
  switch (geo) {
    case kRegular: force_block_kernel<NG, kRegular, SKEL><<<grid, block, 0, s>>>(a, b); break;
    case kStored: force_block_kernel<NG, kStored, SKEL><<<grid, block, 0, s>>>(a, b); break;
    case kTrilinear: force_block_kernel<NG, kTrilinear, SKEL><<<grid, block, 0, s>>>(a, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool SKEL>
hipError_t launch_block_any(int n, int geo, const ForceArgs& a, const BlockArgs& b, hipStream_t s) {
  switch (n) {
    case 2: return launch_block_n<2, SKEL>(geo, a, b, s);
    case 3: return launch_block_n<3, SKEL>(geo, a, b, s);
    case 4: return launch_block_n<4, SKEL>(geo, a, b, s);
    case 5: return launch_block_n<5, SKEL>(geo, a, b, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_force_block(int n, int geo, const ForceArgs& a, const BlockArgs& b, hipStream_t s) {
  return launch_block_any<false>(n, geo, a, b, s);
}

hipError_t launch_force_block_skeleton(int n, int geo, const ForceArgs& a, const BlockArgs& b, hipStream_t s) {
  return launch_block_any<true>(n, geo, a, b, s);
}

}  // namespace semx
