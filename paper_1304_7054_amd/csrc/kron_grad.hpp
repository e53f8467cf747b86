// Gradients of the batched Kronecker action with respect to the shared
// factors, for L = sum_p <dY_p, Y_p>.
//
// 3-D (element (a, b, c) of an operand at a*n^2 + b*n + c, Y(i, j, k) =
// sum A(i, a) B(j, b) C(k, c) X(a, b, c)):
//   dA(i, a) = sum_p sum_{j,k} dY(i, j, k) U(a, j, k),  U = X with B on b and C on c
//   dB(j, b) = sum_p sum_{i,k} dY(i, j, k) V(i, b, k),  V = X with A on a and C on c
//   dC(k, c) = sum_p sum_{i,j} dY(i, j, k) W(i, j, c),  W = X with A on a and B on b
// 2-D (X(u, v) at u*n + v, Y(i, j) = sum A(i, u) B(j, v) X(u, v)):
//   dA(i, u) = sum_p sum_j dY(i, j) Z(u, j),  Z = X with B on v
//   dB(j, v) = sum_p sum_i dY(i, j) W(i, v),  W = X with A on u
// The paper folds transposes into the constant factors once (Section 2.2);
// dX is the forward action with every factor transposed and runs on the
// forward kernels.
//
// Per tile, each factor gradient is one more contraction on the matrix
// cores: the two-factor product of X is formed in registers (two MFMA stages
// and, in 3-D, one lane-group <-> slab exchange) in a layout whose row index
// lines up with dY loaded in a matching layout, and the 16 x 16 product
// dY * T^T accumulates across all tiles a wavefront visits.  Each wavefront
// then writes its 16 x 16 partials; a second kernel sums them in a fixed
// order (deterministic) and folds the diagonal blocks of packed tiles.
#pragma once

#include "kron_kernels.hpp"
#include "kron_staged.hpp"

namespace kron {

// Plain product of two data operands: acc += sum_s a[s] * b[s] on the
// 16x16 instruction of the mode (FP32 or FP64 only).
template <class M>
__device__ __forceinline__ typename M::acc_t mma_data(const typename M::acc_t& a, const typename M::acc_t& b,
                                                      typename M::acc_t acc);
template <>
__device__ __forceinline__ f32x4 mma_data<ModeF32>(const f32x4& a, const f32x4& b, f32x4 acc) {
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma_f32(a[s], b[s], acc);
  return acc;
}
template <>
__device__ __forceinline__ f64x4 mma_data<ModeF64>(const f64x4& a, const f64x4& b, f64x4 acc) {
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma_f64(a[s], b[s], acc);
  return acc;
}

// Loads of a tile in an arbitrary axis assignment: memory axis `LAX` on the
// lane index L, `GAX` on the row-group slots (kmap 0: 4g + s, 1: drow(g, s)),
// `SAX` on the slab index.  Axes are 0 (slow, stride n^2), 1 (n), 2 (1).
template <class M, int N, int Dim>
struct GradLoader {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  static constexpr int Q = Geo<N>::Q;
  static constexpr int E = Dim == 3 ? N * N * N : N * N;
  __device__ static constexpr int stride(int ax) { return Dim == 3 ? (ax == 0 ? N * N : ax == 1 ? N : 1) : (ax == 0 ? N : 1); }
  __device__ static constexpr int opmul(int ax) { return Dim == 3 ? (ax == 0 ? Q * Q : ax == 1 ? Q : 1) : (ax == 0 ? Q : 1); }

  int offL, opL, offG[4], opG[4];
  bool vL, vG[4];

  __device__ __forceinline__ GradLoader(int L, int g, int lax, int gax, int kmap) {
    AxisPart<N, E> pl(L, stride(lax), opmul(lax));
    offL = pl.off; opL = pl.op; vL = pl.valid;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      AxisPart<N, E> pg(kmap == 0 ? 4 * g + s : M::drow(g, s), stride(gax), opmul(gax));
      offG[s] = pg.off; opG[s] = pg.op; vG[s] = pg.valid;
    }
  }

  // one slab (sax < 0: no slab axis, 2-D)
  __device__ __forceinline__ acc_t load(const io_t* P, int64_t rem, int slab, int sax) const {
    int offS = 0, opS = 0;
    bool vS = true;
    if (sax >= 0) {
      AxisPart<N, E> ps(slab, stride(sax), opmul(sax));
      offS = ps.off; opS = ps.op; vS = ps.valid;
    }
    acc_t v;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool ok = vS && vL && vG[s] && (opL + opS + opG[s] < rem);
      v[s] = ok ? in_global(P)[offL + offS + offG[s]] : 0;
    }
    return v;
  }
};

// Per-wavefront accumulation of the factor gradients over its tiles.
// kWhich: bit 0 dA, bit 1 dB, bit 2 dC (3-D).
template <class M, int N>
struct Grad3D {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  using fac_t = typename M::fac_t;
  static constexpr int Q = Geo<N>::Q;
  static constexpr int kOps = Q * Q * Q;
  fac_t fA, fB, fC;  // Mt(L, 4g + s)
  int L, g;

  __device__ __forceinline__ Grad3D(const io_t* A, const io_t* B, const io_t* C, int L_, int g_) : L(L_), g(g_) {
    fA = M::template load_fac<N, false>(A, L, g, 0);
    fB = M::template load_fac<N, false>(B, L, g, 0);
    fC = M::template load_fac<N, false>(C, L, g, 0);
  }

  // Contract the G index of t with factor f (data as MFMA operand B), per
  // slab.  A slab whose slot holds no element is zero before and after (its
  // data, or after swap_rows_slabs the factor row it came from, is zero), so
  // it is skipped.
  __device__ __forceinline__ void stage(const fac_t& f, acc_t (&t)[16]) const {
#pragma unroll
    for (int s = 0; s < 16; ++s)
      if (slot_live<N>(s)) t[s] = M::template db<Geo<N>::kSteps>(f, t[s]);
  }

  // t: rows on (g, r) via drow, slabs s -> slabs = old rows, G slots 4g + s = old slabs
  __device__ __forceinline__ static void swap_rows_slabs(acc_t (&t)[16]) {
    exchange_groups_slabs(t);
    acc_t u[16];
#pragma unroll
    for (int o = 0; o < 16; ++o) Tile3D<M, N, false, false>::regather(t, o, u[o]);
#pragma unroll
    for (int o = 0; o < 16; ++o) t[o] = u[o];
  }

  // acc += sum over slabs of dY(L-row, G) * T(G, L-col) (slabs that hold no
  // element are zero on both sides and skipped)
  __device__ __forceinline__ static void contract(const acc_t (&dy)[16], const acc_t (&t)[16], acc_t& acc) {
#pragma unroll
    for (int s = 0; s < 16; ++s)
      if (slot_live<N>(s)) acc = mma_data<M>(dy[s], t[s], acc);
  }

  // one gradient of one tile.  F = 0 (dA), 1 (dB), 2 (dC).
  template <int F>
  __device__ __forceinline__ void tile(const io_t* Xt, const io_t* dYt, int64_t rem, acc_t& acc) const {
    // X layout: L = the factor's own axis, G = first contracted axis, S = second.
    //   dA: L = a, G = c, S = b;  contract c with C, swap, contract b with B -> (G = j, L = a, S = k)
    //   dB: L = b, G = c, S = a;  contract c with C, swap, contract a with A -> (G = i, L = b, S = k)
    //   dC: L = c, G = b, S = a;  contract b with B, swap, contract a with A -> (G = i, L = c, S = j)
    constexpr int lax = F;
    constexpr int gax = F == 2 ? 1 : 2;
    constexpr int sax = F == 0 ? 1 : 0;
    GradLoader<M, N, 3> lx(L, g, lax, gax, 0);
    acc_t t[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) t[s] = lx.load(Xt, rem, s, sax);
    stage(F == 2 ? fB : fC, t);
    swap_rows_slabs(t);
    stage(F == 0 ? fB : fA, t);
    // dY layout: L = the factor's output index (same axis as `lax`), G = the
    // row index just produced (drow slots), S = the remaining axis.
    //   dA: L = i, G = j, S = k;  dB: L = j, G = i, S = k;  dC: L = k, G = i, S = j
    constexpr int ygax = F == 0 ? 1 : 0;
    constexpr int ysax = F == 2 ? 1 : 2;
    GradLoader<M, N, 3> ly(L, g, lax, ygax, 1);
    acc_t dy[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) dy[s] = ly.load(dYt, rem, s, ysax);
    contract(dy, t, acc);
  }
};

template <class M, int N>
struct Grad2D {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  using fac_t = typename M::fac_t;
  static constexpr int Q = Geo<N>::Q;
  static constexpr int kOps = Q * Q;
  fac_t fA, fB;
  int L, g;

  __device__ __forceinline__ Grad2D(const io_t* A, const io_t* B, int L_, int g_) : L(L_), g(g_) {
    fA = M::template load_fac<N, false>(A, L, g, 0);
    fB = M::template load_fac<N, false>(B, L, g, 0);
  }

  // F = 0 (dA): X (L = u, G = v), contract v with B -> (G = j, L = u); dY (L = i, G = j)
  // F = 1 (dB): X (L = v, G = u), contract u with A -> (G = i, L = v); dY (L = j, G = i)
  template <int F>
  __device__ __forceinline__ void tile(const io_t* Xt, const io_t* dYt, int64_t rem, acc_t& acc) const {
    constexpr int lax = F, gax = 1 - F;
    GradLoader<M, N, 2> lx(L, g, lax, gax, 0);
    acc_t t = M::template db<Geo<N>::kSteps>(F == 0 ? fB : fA, lx.load(Xt, rem, 0, -1));
    GradLoader<M, N, 2> ly(L, g, lax, gax, 1);
    acc = mma_data<M>(ly.load(dYt, rem, 0, -1), t, acc);
  }
};

constexpr int kGradBlock = 256;

// FP32: X and dY of a tile are copied once into the wavefront's LDS (16-byte
// coalesced loads), and the six operand layouts the three gradients need are
// read from there (one address register per row-group slot plus immediate
// offsets).  FP64 tiles would not fit, so FP64 reads global memory directly.
template <class M, int N>
constexpr bool kGradStaged = sizeof(typename M::io_t) == 4;

template <class M, int N>
struct Grad3DStaged {
  using io_t = typename M::io_t;
  using acc_t = typename M::acc_t;
  using fac_t = typename M::fac_t;
  using G = TileGeom<N, 3>;
  static constexpr int Q = Geo<N>::Q;
  static constexpr int kOps = Q * Q * Q;
  static constexpr int E = G::E;
  static constexpr int kElems = kOps * E;
  static constexpr int kSlice = (kElems + kStagePad + 7) / 8 * 8;
  fac_t fA, fB, fC;
  int L, g;

  __device__ __forceinline__ Grad3DStaged(const io_t* A, const io_t* B, const io_t* C, int L_, int g_)
      : L(L_), g(g_) {
    fA = M::template load_fac<N, false>(A, L, g, 0);
    fB = M::template load_fac<N, false>(B, L, g, 0);
    fC = M::template load_fac<N, false>(C, L, g, 0);
  }

  template <int SAX>
  __device__ __forceinline__ static acc_t read(const io_t* lds, const LaneSlots<N, 3>& ls, int slab) {
    AxisPart<N, E> ps(slab, G::stride(SAX), G::opmul(SAX));
    acc_t v = acc_t{0, 0, 0, 0};
    if (!ps.valid) return v;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float x = in_lds(lds)[ls.base[s] + ps.off];
      v[s] = ls.ok[s] ? x : 0.f;
    }
    return v;
  }

  // F = 0 (dA), 1 (dB), 2 (dC); same layouts as Grad3D::tile.
  template <int F>
  __device__ __forceinline__ void tile(const io_t* ldsX, const io_t* ldsY, acc_t& acc) const {
    constexpr int lax = F;
    constexpr int gax = F == 2 ? 1 : 2;
    constexpr int sax = F == 0 ? 1 : 0;
    constexpr int ygax = F == 0 ? 1 : 0;
    constexpr int ysax = F == 2 ? 1 : 2;
    const LaneSlots<N, 3> lx(L, lax, g, gax, false);
    acc_t t[16];
    // slabs whose slot holds no element stay zero through every step and are
    // skipped (as in Grad3D)
#pragma unroll
    for (int s = 0; s < 16; ++s)
      t[s] = slot_live<N>(s) ? M::template db<Geo<N>::kSteps>(F == 2 ? fB : fC, read<sax>(ldsX, lx, s)) : acc_t{0, 0, 0, 0};
    Grad3D<M, N>::swap_rows_slabs(t);
#pragma unroll
    for (int s = 0; s < 16; ++s)
      if (slot_live<N>(s)) t[s] = M::template db<Geo<N>::kSteps>(F == 0 ? fB : fA, t[s]);
    const LaneSlots<N, 3> ly(L, lax, g, ygax, M::drow(0, 1) != 1);
#pragma unroll
    for (int s = 0; s < 16; ++s)
      if (slot_live<N>(s)) acc = mma_data<M>(read<ysax>(ldsY, ly, s), t[s], acc);
  }
};

// Partials: ws[(wave * 3 + f) * 256 + row * 16 + col] holds wavefront `wave`'s
// 16 x 16 tile of factor f's gradient (row = drow(g, r), col = L).
template <class M, int N, int Dim>
__global__ __launch_bounds__(kGradBlock) void kron_grad_partial_kernel(
    const typename M::io_t* __restrict__ A, const typename M::io_t* __restrict__ B,
    const typename M::io_t* __restrict__ C, const typename M::io_t* __restrict__ X,
    const typename M::io_t* __restrict__ dY, typename M::elem_t* __restrict__ ws, int64_t batch,
    int64_t ntiles, int which) {
  using acc_t = typename M::acc_t;
  using T = typename M::elem_t;
  using io_t = typename M::io_t;
  const int l = threadIdx.x & 63, L = l & 15, g = l >> 4;
  const int64_t wave = ((int64_t)blockIdx.x * kGradBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kGradBlock) >> 6;
  acc_t acc[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) acc[f] = acc_t{0, 0, 0, 0};
  if constexpr (Dim == 3 && kGradStaged<M, N>) {
    using GS = Grad3DStaged<M, N>;
    __shared__ __attribute__((aligned(16))) io_t slices[kGradBlock / kWave][2][GS::kSlice];
    io_t* sliceX = slices[threadIdx.x >> 6][0];
    io_t* sliceY = slices[threadIdx.x >> 6][1];
    const GS gr(A, B, C, L, g);
    for (int64_t t = wave; t < ntiles; t += nwaves) {
      const int64_t rem = batch - t * GS::kOps;
      const int count = (int)((rem < GS::kOps ? rem : GS::kOps) * GS::E);
      const io_t* Xt = X + t * GS::kElems;
      const io_t* dYt = dY + t * GS::kElems;
      io_t* ldsX = stage_base(sliceX, Xt);
      io_t* ldsY = stage_base(sliceY, dYt);
      wave_sync_lds();
      zero_fill(ldsX, count, GS::kElems, l);
      zero_fill(ldsY, count, GS::kElems, l);
      copy_in(Xt, ldsX, count, l);
      copy_in(dYt, ldsY, count, l);
      wave_sync_lds();
      if (which & 1) gr.template tile<0>(ldsX, ldsY, acc[0]);
      if (which & 2) gr.template tile<1>(ldsX, ldsY, acc[1]);
      if (which & 4) gr.template tile<2>(ldsX, ldsY, acc[2]);
    }
  } else if constexpr (Dim == 3) {
    using G3 = Grad3D<M, N>;
    constexpr int64_t step = (int64_t)G3::kOps * N * N * N;
    const G3 gr(A, B, C, L, g);
    for (int64_t t = wave; t < ntiles; t += nwaves) {
      const int64_t rem = batch - t * G3::kOps;
      if (which & 1) gr.template tile<0>(X + t * step, dY + t * step, rem, acc[0]);
      if (which & 2) gr.template tile<1>(X + t * step, dY + t * step, rem, acc[1]);
      if (which & 4) gr.template tile<2>(X + t * step, dY + t * step, rem, acc[2]);
    }
  } else {
    using G2 = Grad2D<M, N>;
    constexpr int64_t step = (int64_t)G2::kOps * N * N;
    const G2 gr(A, B, L, g);
    for (int64_t t = wave; t < ntiles; t += nwaves) {
      const int64_t rem = batch - t * G2::kOps;
      if (which & 1) gr.template tile<0>(X + t * step, dY + t * step, rem, acc[0]);
      if (which & 2) gr.template tile<1>(X + t * step, dY + t * step, rem, acc[1]);
    }
  }
#pragma unroll
  for (int f = 0; f < 3; ++f)
#pragma unroll
    for (int r = 0; r < 4; ++r) ws[(wave * 3 + f) * 256 + M::drow(g, r) * 16 + L] = (T)acc[f][r];
}

// ---- fused 3-D backward for n = 16 (one operand per tile) ----------------------
//
// One 256-thread workgroup per tile at a time: the four wavefronts copy X and
// dY of the tile into LDS together, then wavefronts 0, 1, 2 each accumulate
// one factor gradient (dA, dB, dC) and wavefront 3 computes dX, the forward
// action with every factor transposed, and stores it.  Each array is read
// from HBM once and dX written once.  In LDS, rows of 16 elements sit at a
// pitch of 20 and slabs at a pitch of 324 elements: rows stay 16-byte
// aligned for the copies, and the reads along the slow axes, which the
// gradient layouts need, fall on at most 4 lanes per bank instead of 16.
struct Pad16 {
  static constexpr int P1 = 20;
  static constexpr int P0 = 16 * P1 + 4;
  static constexpr int kElems = 16 * P0;
  __device__ static constexpr int stride(int ax) { return ax == 0 ? P0 : ax == 1 ? P1 : 1; }
};

// A tile (4096 elements, 16-byte aligned) moves into its padded LDS image
// in two steps, so that the loads of the next tile can be in flight while
// the current one is computed: every thread loads 4 of the 1024 16-byte
// vectors into registers, and later writes them to their padded places.
__device__ __forceinline__ void load_tile16(const float* __restrict__ src, f32x4 (&r)[4], int tid) {
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = Mem<float>::load4(src + 4 * (tid + 256 * k));
}
__device__ __forceinline__ void store_tile16(const f32x4 (&r)[4], float* lds, int tid) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = 4 * (tid + 256 * k);
    const int off = (e >> 8) * Pad16::P0 + ((e >> 4) & 15) * Pad16::P1 + (e & 15);
    *in_lds(reinterpret_cast<f32x4*>(lds + off)) = r[k];
  }
}

// One factor gradient of one tile from the padded images (same layouts and
// steps as Grad3D::tile).
template <class M, int F>
__device__ __forceinline__ void grad16_tile(const float* ldsX, const float* ldsY, const typename M::fac_t& fA,
                                            const typename M::fac_t& fB, const typename M::fac_t& fC, int L, int g,
                                            typename M::acc_t& acc) {
  using acc_t = typename M::acc_t;
  constexpr int lax = F, gax = F == 2 ? 1 : 2, sax = F == 0 ? 1 : 0;
  constexpr int ygax = F == 0 ? 1 : 0, ysax = F == 2 ? 1 : 2;
  int bx[4], by[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    bx[q] = L * Pad16::stride(lax) + (4 * g + q) * Pad16::stride(gax);
    by[q] = L * Pad16::stride(lax) + M::drow(g, q) * Pad16::stride(ygax);
  }
  acc_t t[16];
  if constexpr (gax == 2) {
    // the four slots 4g .. 4g + 3 are consecutive, 16-byte aligned elements
#pragma unroll
    for (int sl = 0; sl < 16; ++sl) t[sl] = *in_lds(reinterpret_cast<const acc_t*>(ldsX + bx[0] + sl * Pad16::stride(sax)));
  } else {
#pragma unroll
    for (int sl = 0; sl < 16; ++sl)
#pragma unroll
      for (int q = 0; q < 4; ++q) t[sl][q] = in_lds(ldsX)[bx[q] + sl * Pad16::stride(sax)];
  }
#pragma unroll
  for (int sl = 0; sl < 16; ++sl) t[sl] = M::db(F == 2 ? fB : fC, t[sl]);
  Grad3D<M, 16>::swap_rows_slabs(t);
#pragma unroll
  for (int sl = 0; sl < 16; ++sl) t[sl] = M::db(F == 0 ? fB : fA, t[sl]);
  // four independent accumulators (slab mod 4) keep the matrix-core pipe fed
  // instead of one dependent chain of 64 products; summed in a fixed order
  acc_t part[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) part[j] = acc_t{0.f, 0.f, 0.f, 0.f};
  if constexpr (ysax == 2) {
    // four consecutive slabs of one slot are consecutive, 16-byte aligned elements
#pragma unroll
    for (int s4 = 0; s4 < 16; s4 += 4) {
      acc_t quad[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) quad[q] = *in_lds(reinterpret_cast<const acc_t*>(ldsY + by[q] + s4));
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const acc_t dy = acc_t{quad[0][j], quad[1][j], quad[2][j], quad[3][j]};
        part[j] = mma_data<M>(dy, t[s4 + j], part[j]);
      }
    }
  } else {
#pragma unroll
    for (int sl = 0; sl < 16; ++sl) {
      acc_t dy;
#pragma unroll
      for (int q = 0; q < 4; ++q) dy[q] = in_lds(ldsY)[by[q] + sl * Pad16::stride(ysax)];
      part[sl & 3] = mma_data<M>(dy, t[sl], part[sl & 3]);
    }
  }
  acc += (part[0] + part[1]) + (part[2] + part[3]);
}

// Partials: ws[(block * 3 + f) * 256 + row * 16 + col], as the per-wavefront
// kernel writes them (the reduction kernel is shared).  `which` bit f asks
// for factor f's gradient; dX may be null.
__global__ __launch_bounds__(kGradBlock) __attribute__((amdgpu_waves_per_eu(2))) void kron3d_backward16_kernel(
    const float* __restrict__ A, const float* __restrict__ B, const float* __restrict__ C,
    const float* __restrict__ X, const float* __restrict__ dY, float* __restrict__ dX, float* __restrict__ ws,
    int64_t ntiles, int which) {
  using M = ModeF32;
  using acc_t = M::acc_t;
  __shared__ __attribute__((aligned(16))) float sX[Pad16::kElems];
  __shared__ __attribute__((aligned(16))) float sY[Pad16::kElems];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, L = l & 15, g = l >> 4;
  const bool grads = which != 0;
  const M::fac_t fA = M::load_fac<16, false>(A, L, g, 0);
  const M::fac_t fB = M::load_fac<16, false>(B, L, g, 0);
  const M::fac_t fC = M::load_fac<16, false>(C, L, g, 0);
  const Tile3D<M, 16, false, true, true> fwd(A, B, C, L, g);
  acc_t acc[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) acc[f] = acc_t{0.f, 0.f, 0.f, 0.f};
  int role = w;  // rotates by one per tile, so every SIMD takes every role in turn
  f32x4 px[4], py[4];  // the next tile's X and dY, in flight while the current tile is computed
  if (blockIdx.x < ntiles) {
    if (grads) load_tile16(X + blockIdx.x * 4096, px, tid);
    load_tile16(dY + blockIdx.x * 4096, py, tid);
  }
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x, role = (role + 1) & 3) {
    __syncthreads();  // every wavefront is done with the previous tile's images
    if (grads) store_tile16(px, sX, tid);
    store_tile16(py, sY, tid);
    __syncthreads();
    const int64_t tn = t + gridDim.x;
    if (tn < ntiles) {
      if (grads) load_tile16(X + tn * 4096, px, tid);
      load_tile16(dY + tn * 4096, py, tid);
    }
    if (role < 3 ? !((which >> role) & 1) : dX == nullptr) continue;
    if (role == 0) grad16_tile<M, 0>(sX, sY, fA, fB, fC, L, g, acc[0]);
    else if (role == 1) grad16_tile<M, 1>(sX, sY, fA, fB, fC, L, g, acc[1]);
    else if (role == 2) grad16_tile<M, 2>(sX, sY, fA, fB, fC, L, g, acc[2]);
    else {
      // slab a on the slow axis, L on the middle axis, slots 4g + s on the fast axis
      acc_t v[16];
#pragma unroll
      for (int a = 0; a < 16; ++a) {
        v[a] = *in_lds(reinterpret_cast<const f32x4*>(sY + a * Pad16::P0 + L * Pad16::P1 + 4 * g));
        fwd.stage12(v[a]);
      }
      fwd.stage3(v);
      float* dXt = dX + t * 4096;
#pragma unroll
      for (int i = 0; i < 16; ++i) Mem<float>::store4(dXt + i * 256 + L * 16 + 4 * g, v[i]);
    }
  }
  // the four wavefronts' partials, summed in wavefront order through LDS
  __syncthreads();
  float* red = sX;  // 4 x 3 x 256 floats
#pragma unroll
  for (int f = 0; f < 3; ++f)
#pragma unroll
    for (int r = 0; r < 4; ++r) in_lds(red)[(w * 3 + f) * 256 + M::drow(g, r) * 16 + L] = acc[f][r];
  __syncthreads();
  for (int e = tid; e < 3 * 256; e += kGradBlock) {
    const int f = e >> 8, idx = e & 255;
    float sum = 0.f;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) sum += in_lds(red)[(ww * 3 + f) * 256 + idx];
    ws[((int64_t)blockIdx.x * 3 + f) * 256 + idx] = sum;
  }
}

// dM(i, j) = sum over the partial tiles and over the Q diagonal blocks of
// each (logical index q*n + i sits in slot slot_of(q*n + i)).  One workgroup
// per entry (i, j) of each factor: thread t sums partials t, t + 256, ... in
// order in FP64, then a fixed-shape tree over the 256 thread sums finishes
// the entry, so the result does not depend on timing.  Output column-major
// (i + n*j).
template <typename io_t, typename T, int N>
__global__ __launch_bounds__(kGradBlock) void kron_grad_reduce_kernel(const T* __restrict__ ws, int64_t nparts,
                                                                      io_t* __restrict__ dA, io_t* __restrict__ dB,
                                                                      io_t* __restrict__ dC) {
  constexpr int Q = Geo<N>::Q;
  const int f = blockIdx.x / (N * N), e = blockIdx.x % (N * N);
  io_t* out = f == 0 ? dA : f == 1 ? dB : dC;
  if (out == nullptr) return;
  const int i = e % N, j = e / N;
  double s = 0.0;
  for (int64_t w = threadIdx.x; w < nparts; w += kGradBlock) {
    const T* tile = ws + (w * 3 + f) * 256;
#pragma unroll
    for (int q = 0; q < Q; ++q) s += (double)tile[slot_of<N>(q * N + i) * 16 + slot_of<N>(q * N + j)];
  }
  __shared__ double red[kGradBlock];
  red[threadIdx.x] = s;
  __syncthreads();
#pragma unroll
  for (int h = kGradBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i + N * j] = (io_t)red[0];
}

}  // namespace kron
