// FP32 element internal-force kernel f = -K u over element patches.
//
// A patch is a short chain of elements that share nodes (built on the host
// from the global-to-local map).  One workgroup owns one patch:
//   1. the patch's unique global nodes of u are copied into LDS; they are
//      stored as runs of consecutive global indices, a wavefront copies
//      whole runs (several in flight), so neighbouring lanes read
//      neighbouring 12-byte nodes;
//   2. the elements of the chain are computed in rounds of EPR elements side
//      by side with the same fused traversal as the per-element kernel
//      (gather from the patch tile through a 16-bit local index, forward
//      contractions with D, inverse-Jacobian map, isotropic stress, weighted
//      fluxes, transpose contractions; Sec. II-B, Sec. IV-D), and each
//      element's forces are added into a patch force tile in LDS with LDS
//      atomics, so nodes shared inside the chain are summed there.  Every
//      per-element input of the patch (local indices, lambda', mu', geometry
//      words) is requested once, before the first round, so the rounds run
//      without waiting on memory;
//   3. every patch node is written back once.  Coloured assembly: patches of
//      one colour share no node, so a plain read-modify-write is race-free,
//      and a node's first touch in colour order stores without reading
//      (the force vector needs no clearing).  Atomic assembly: nodes that
//      only this patch touches are stored, the others take one FP32 atomic
//      add per component.
// This is the graph-coloured versus atomic assembly of Sec. IV-C at patch
// granularity: each launch then touches whole rows of nodes instead of the
// scattered single-element segments of a per-element colour class.
#include "elem_common.hpp"

namespace semx {
namespace {

constexpr int kRunsPerPass = 8;  // runs a wavefront moves per pass (loads in flight)

__device__ __forceinline__ int run_len(int d) { return d & ((1 << kRunLenBits) - 1); }
__device__ __forceinline__ int run_off(int d) { return (d >> kRunLenBits) & ((1 << kRunLenBits) - 1); }

// Launch shape: EPR elements of a patch are computed side by side (one
// n^3-lane group each), so a workgroup has about 256 lanes; a chain of up to
// kPatchMaxElems elements takes MAXR rounds.
template <int NG>
struct PShape {
  static constexpr int N3 = Shape<NG>::N3;
  static constexpr int BLK = Shape<NG>::BLK;
  static constexpr int EPR = BLK >= 256 ? 1 : 256 / BLK;
  static constexpr int WG = EPR * BLK;
  static constexpr int MAXR = (kPatchMaxElems + EPR - 1) / EPR;
  static constexpr int NW = WG / 64;  // wavefronts
};

template <int NG, int GEO, bool ATOMIC>
__global__ __launch_bounds__(PShape<NG>::WG) void force_patch_kernel(PatchArgs pa) {
  using S = PShape<NG>;
  constexpr int N3 = S::N3, BLK = S::BLK, EPR = S::EPR, WG = S::WG, MAXR = S::MAXR, NW = S::NW;
  constexpr int GW = GEO == kTrilinear ? 24 : 9;  // per-element geometry words
  extern __shared__ float s_dyn[];
  __shared__ float s_u[EPR][3 * N3];
  __shared__ float s_q[EPR][9 * N3];
  __shared__ float s_D[NG * NG];
  __shared__ int s_pos[kPatchMaxElems];
  __shared__ float s_geo[kPatchMaxElems * GW];
  const ForceArgs& a = pa.fa;

  const int np = (int)a.count;
  const int grp = xcd_group(np);
  if (grp >= np) return;  // uniform over the block
  const int p = (int)a.pos0 + grp;
  const int e0 = pa.pe_off[p], ne = pa.pe_off[p + 1] - e0;
  const int r0 = pa.pr_off[p], nr = pa.pr_off[p + 1] - r0;
  const int MN = pa.maxnodes, MR = pa.maxruns;
  float* sux = s_dyn;
  float* suy = sux + MN;
  float* suz = suy + MN;
  float* sfx = suz + MN;
  float* sfy = sfx + MN;
  float* sfz = sfy + MN;
  int* srs = reinterpret_cast<int*>(sfz + MN);
  int* srd = srs + MR;

  const int t = threadIdx.x;
  const int wave = t / 64, lane = t % 64;
  const int sub = t / BLK;  // element slot inside a round
  const int pl = t % BLK;
  const bool act = pl < N3;
  const int pp = act ? pl : 0;
  const int i = pp % NG, j = (pp / NG) % NG, k = pp / (NG * NG);
  const int model = blockIdx.y;
  const float* __restrict__ u = a.u + (size_t)model * a.nglob * 3;
  float* f = a.f + (size_t)model * a.nglob * 3;
  const float* __restrict__ mat = a.mat + (size_t)model * a.nspec * 2 * N3;
  float rx = 0.f, ry = 0.f, rz = 0.f;  // reference coordinates (trilinear path)
  if constexpr (GEO == kTrilinear) {
    rx = a.xi[i];
    ry = a.xi[j];
    rz = a.xi[k];
  }

  // 0. element positions, runs, D
  if (t < ne) s_pos[t] = pa.pe_pos[e0 + t];
  for (int r = t; r < nr; r += WG) {
    srs[r] = pa.runs[2 * (size_t)(r0 + r)];
    srd[r] = pa.runs[2 * (size_t)(r0 + r) + 1];
  }
  if (t < NG * NG) s_D[t] = a.D[t];
  __syncthreads();

  // 1. everything the patch reads from memory, issued together: element
  //    geometry words -> LDS, each lane's streams for all its rounds ->
  //    registers, u of the patch nodes -> LDS (a wave copies whole runs)
  if constexpr (GEO != kStored) {
    const float* gsrc = GEO == kTrilinear ? a.tri : a.gam_el;
    for (int q = t; q < ne * GW; q += WG) s_geo[q] = gsrc[(size_t)s_pos[q / GW] * GW + q % GW];
  }
  int L[MAXR];
  float LW[MAXR], MW[MAXR];
  float G[9];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    const int m = r * EPR + sub;
    L[r] = 0;
    LW[r] = MW[r] = 0.0f;
    if (m < ne) {
      const int pos = s_pos[m];
      L[r] = pa.lidx[(size_t)(e0 + m) * N3 + pp];
      LW[r] = ldnt(mat + (size_t)pos * 2 * N3 + pp);
      MW[r] = ldnt(mat + (size_t)pos * 2 * N3 + N3 + pp);
    }
  }
  if constexpr (GEO == kStored) {
    const float* gp = a.gam_pt + (size_t)s_pos[sub < ne ? sub : 0] * 9 * N3 + pp;
#pragma unroll
    for (int d = 0; d < 9; ++d) G[d] = ldnt(gp + d * N3);
  }
  // each wave takes U runs at a time: all their loads, then the LDS stores
  for (int rb = wave; rb < nr; rb += NW * kRunsPerPass) {
    float x[kRunsPerPass], y[kRunsPerPass], z[kRunsPerPass];
    int dst[kRunsPerPass];
#pragma unroll
    for (int uu = 0; uu < kRunsPerPass; ++uu) {
      const int r = rb + uu * NW;
      dst[uu] = -1;
      if (r < nr) {
        const int d = srd[r];
        if (lane < run_len(d)) {
          const float* up = u + 3 * (size_t)(srs[r] + lane);
          x[uu] = up[0];
          y[uu] = up[1];
          z[uu] = up[2];
          dst[uu] = run_off(d) + lane;
        }
      }
    }
#pragma unroll
    for (int uu = 0; uu < kRunsPerPass; ++uu) {
      if (dst[uu] >= 0) {
        sux[dst[uu]] = x[uu];
        suy[dst[uu]] = y[uu];
        suz[dst[uu]] = z[uu];
        sfx[dst[uu]] = 0.0f;
        sfy[dst[uu]] = 0.0f;
        sfz[dst[uu]] = 0.0f;
      }
    }
    // the rare run longer than a wavefront
#pragma unroll
    for (int uu = 0; uu < kRunsPerPass; ++uu) {
      const int r = rb + uu * NW;
      if (r < nr) {
        const int d = srd[r], len = run_len(d), off = run_off(d);
        for (int q = lane + 64; q < len; q += 64) {
          const float* up = u + 3 * (size_t)(srs[r] + q);
          sux[off + q] = up[0];
          suy[off + q] = up[1];
          suz[off + q] = up[2];
          sfx[off + q] = 0.0f;
          sfy[off + q] = 0.0f;
          sfz[off + q] = 0.0f;
        }
      }
    }
  }
  __syncthreads();

  // 2. rounds of EPR elements
  const int nround = (ne + EPR - 1) / EPR;
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    if (r >= nround) break;  // uniform over the block
    const int m = r * EPR + sub;
    const bool live = m < ne;
    if (live && act) {
      const int l = L[r];
      s_u[sub][pp] = sux[l];
      s_u[sub][N3 + pp] = suy[l];
      s_u[sub][2 * N3 + pp] = suz[l];
    }
    float Gn[9];
    if constexpr (GEO == kStored) {  // next round's Gamma
      const int mn = (r + 1) * EPR + sub;
      if (r + 1 < nround && mn < ne) {
        const float* gp = a.gam_pt + (size_t)s_pos[mn] * 9 * N3 + pp;
#pragma unroll
        for (int d = 0; d < 9; ++d) Gn[d] = ldnt(gp + d * N3);
      }
    }
    __syncthreads();
    if (live) {
      float du[3][3];
      ref_grad<NG>(s_u[sub], s_D, i, j, k, du);
      float Mg[9], scale, det;
      geom_map_from<GEO>(s_geo + m * GW, G, rx, ry, rz, Mg, scale, det);
      float gr[3][3];
      apply_map(du, Mg, gr);
      stress_flux(gr, LW[r], MW[r], scale, Mg, s_q[sub], N3, pp, act);
    }
    __syncthreads();
    float F[3] = {0.0f, 0.0f, 0.0f};
    if (live) ref_div<NG>(s_q[sub], s_D, i, j, k, F);
    // the slots of a round add in a fixed order (neighbouring elements of a
    // chain share nodes), so every node's sum is formed in one order and the
    // result is bitwise reproducible
#pragma unroll
    for (int s2 = 0; s2 < EPR; ++s2) {
      if (s2 > 0) __syncthreads();
      if (sub == s2 && live && act) {
        const int l = L[r];
        atomicAdd(sfx + l, F[0]);
        atomicAdd(sfy + l, F[1]);
        atomicAdd(sfz + l, F[2]);
      }
    }
    if constexpr (GEO == kStored) {
#pragma unroll
      for (int d = 0; d < 9; ++d) G[d] = Gn[d];
    }
  }
  __syncthreads();

  // 3. write the patch nodes back, a wave per run (run flags are uniform);
  //    U runs at a time: the reads of the read-modify-writes first
  for (int rb = wave; rb < nr; rb += NW * kRunsPerPass) {
    float ox[kRunsPerPass], oy[kRunsPerPass], oz[kRunsPerPass];
#pragma unroll
    for (int uu = 0; uu < kRunsPerPass; ++uu) {
      const int r = rb + uu * NW;
      ox[uu] = oy[uu] = oz[uu] = 0.0f;
      if constexpr (!ATOMIC) {
        if (r < nr) {
          const int d = srd[r];
          if (lane < run_len(d) && !(d & kRunFirst)) {
            const float* fp = f + 3 * (size_t)(srs[r] + lane);
            ox[uu] = fp[0];
            oy[uu] = fp[1];
            oz[uu] = fp[2];
          }
        }
      }
    }
#pragma unroll
    for (int uu = 0; uu < kRunsPerPass; ++uu) {
      const int r = rb + uu * NW;
      if (r < nr) {
        const int d = srd[r], len = run_len(d), off = run_off(d);
        for (int q = lane; q < len; q += 64) {
          float* fp = f + 3 * (size_t)(srs[r] + q);
          const float x = sfx[off + q], y = sfy[off + q], z = sfz[off + q];
          if constexpr (!ATOMIC) {
            float bx = ox[uu], by = oy[uu], bz = oz[uu];
            if (q >= 64 && !(d & kRunFirst)) {  // beyond the first wavefront's reads
              bx = fp[0];
              by = fp[1];
              bz = fp[2];
            } else if (q >= 64) {
              bx = by = bz = 0.0f;
            }
            fp[0] = bx + x;
            fp[1] = by + y;
            fp[2] = bz + z;
          } else {
            if (d & kRunExclusive) {
              fp[0] = x;
              fp[1] = y;
              fp[2] = z;
            } else {
              unsafeAtomicAdd(fp + 0, x);
              unsafeAtomicAdd(fp + 1, y);
              unsafeAtomicAdd(fp + 2, z);
            }
          }
        }
      }
    }
  }
}

template <int NG>
constexpr size_t static_lds() {
  return sizeof(float) * (12 * PShape<NG>::EPR * Shape<NG>::N3 + NG * NG + kPatchMaxElems * (1 + 24));
}

template <int NG, int GEO, bool ATOMIC>
hipError_t launch_one(const PatchArgs& a, hipStream_t s) {
  const int64_t np = a.fa.count;
  const int64_t nb = ((np + kNumXcd - 1) / kNumXcd) * kNumXcd;
  const size_t dyn = sizeof(float) * (6 * (size_t)a.maxnodes + 2 * (size_t)a.maxruns);
  dim3 grid((unsigned)nb, (unsigned)a.fa.nmodels), block(PShape<NG>::WG);
  force_patch_kernel<NG, GEO, ATOMIC><<<grid, block, dyn, s>>>(a);
  return hipGetLastError();
}

template <int NG>
hipError_t launch_n(int geo, bool atomic, const PatchArgs& a, hipStream_t s) {
  if (a.fa.count <= 0) return hipSuccess;
  if (a.maxnodes > kPatchMaxNodes || a.maxnodes <= 0 || a.maxruns <= 0) return hipErrorInvalidValue;
  switch (geo) {
    case kRegular:
      return atomic ? launch_one<NG, kRegular, true>(a, s) : launch_one<NG, kRegular, false>(a, s);
    case kStored:
      return atomic ? launch_one<NG, kStored, true>(a, s) : launch_one<NG, kStored, false>(a, s);
    case kTrilinear:
      return atomic ? launch_one<NG, kTrilinear, true>(a, s) : launch_one<NG, kTrilinear, false>(a, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

size_t patch_lds_bytes(int n, int maxnodes, int maxruns) {
  size_t st = 0;
  switch (n) {
    case 2: st = static_lds<2>(); break;
    case 3: st = static_lds<3>(); break;
    case 4: st = static_lds<4>(); break;
    case 5: st = static_lds<5>(); break;
    case 6: st = static_lds<6>(); break;
    case 7: st = static_lds<7>(); break;
    case 8: st = static_lds<8>(); break;
    case 9: st = static_lds<9>(); break;
    default: return (size_t)-1;  // no patch kernel for this order
  }
  return st + sizeof(float) * (6 * (size_t)maxnodes + 2 * (size_t)maxruns);
}

hipError_t launch_force_patch(int n, int geo, bool atomic, const PatchArgs& a, hipStream_t s) {
  switch (n) {
    case 2: return launch_n<2>(geo, atomic, a, s);
    case 3: return launch_n<3>(geo, atomic, a, s);
    case 4: return launch_n<4>(geo, atomic, a, s);
    case 5: return launch_n<5>(geo, atomic, a, s);
    case 6: return launch_n<6>(geo, atomic, a, s);
    case 7: return launch_n<7>(geo, atomic, a, s);
    case 8: return launch_n<8>(geo, atomic, a, s);
    case 9: return launch_n<9>(geo, atomic, a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace semx
