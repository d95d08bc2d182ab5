// Device building blocks: complex arithmetic, LDS-resident Stockham FFT,
// real<->complex packing, deterministic FP64 reductions, and the pointwise
// constitutive law in closed form.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spff {

template <typename real> struct CplxOf;
template <> struct CplxOf<float> { using type = float2; };
template <> struct CplxOf<double> { using type = double2; };
template <typename real> using cplx = typename CplxOf<real>::type;

template <typename V> __device__ __forceinline__ V mk(decltype(V::x) a, decltype(V::x) b) {
  V r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return mk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return mk<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cconj(V a) { return mk<V>(a.x, -a.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return mk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// i * a and -i * a
template <typename V> __device__ __forceinline__ V cmuli(V a) { return mk<V>(-a.y, a.x); }
template <typename V> __device__ __forceinline__ V cmulni(V a) { return mk<V>(a.y, -a.x); }
template <typename V> __device__ __forceinline__ V cscale(V a, decltype(V::x) s) { return mk<V>(a.x * s, a.y * s); }

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

// ---------------------------------------------------------------------------
// Stockham autosort FFT on `ntrans` transforms of length M (power of two)
// held in LDS, transform t at buf + t*stride.  A pass with sub-transform size
// Ns and radix Rd (2, 4 or 8):
//   j in [0, M/Rd), k = j mod Ns
//   v_r = x[j + r M/Rd] * w_{Ns Rd}^{r k}          (twiddle)
//   v'  = DFT_Rd(v)
//   y[(j - k) Rd + k + s Ns] = v'_s
// Each pass reads its inputs into registers, synchronises, then writes in
// place (chunks of whole transforms, at most T*MAXE elements per chunk).
// tw holds the (M*twmul)-th roots of unity exp(-2 pi i e/(M twmul)); a
// butterfly loads w^k (and w^4k for radix 8) and forms the other powers by
// products (at most three chained).  The inverse (INV) uses conjugates and is
// unnormalised.  Requires M <= blockDim.x * MAXE.
// ---------------------------------------------------------------------------
template <bool INV, typename V>
__device__ __forceinline__ void bfly4(V& v0, V& v1, V& v2, V& v3) {
  V a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), d = csub(v1, v3);
  V a3 = INV ? cmuli(d) : cmulni(d);
  v0 = cadd(a0, a2);
  v1 = cadd(a1, a3);
  v2 = csub(a0, a2);
  v3 = csub(a1, a3);
}

// 8-point DFT in place (natural order in and out): two 4-point DFTs of the
// even and odd inputs, combined with w8^s.
template <bool INV, typename V>
__device__ __forceinline__ void bfly8(V* v) {
  using T = decltype(V::x);
  const T h = T(0.70710678118654752440084436210485);
  V a0 = v[0], a1 = v[2], a2 = v[4], a3 = v[6];
  V b0 = v[1], b1 = v[3], b2 = v[5], b3 = v[7];
  bfly4<INV>(a0, a1, a2, a3);
  bfly4<INV>(b0, b1, b2, b3);
  if (INV) {
    b1 = mk<V>((b1.x - b1.y) * h, (b1.x + b1.y) * h);
    b2 = cmuli(b2);
    b3 = mk<V>(-(b3.x + b3.y) * h, (b3.x - b3.y) * h);
  } else {
    b1 = mk<V>((b1.x + b1.y) * h, (b1.y - b1.x) * h);
    b2 = cmulni(b2);
    b3 = mk<V>((b3.y - b3.x) * h, -(b3.x + b3.y) * h);
  }
  v[0] = cadd(a0, b0);
  v[4] = csub(a0, b0);
  v[1] = cadd(a1, b1);
  v[5] = csub(a1, b1);
  v[2] = cadd(a2, b2);
  v[6] = csub(a2, b2);
  v[3] = cadd(a3, b3);
  v[7] = csub(a3, b3);
}

template <typename real, bool INV, int MAXE, int RD>
__device__ __forceinline__ void stockham_pass(cplx<real>* buf, int logM, int logNs, int ntrans, int stride,
                                              const cplx<real>* __restrict__ tw, int twmul, int tpc) {
  using V = cplx<real>;
  constexpr int LR = RD == 8 ? 3 : (RD == 4 ? 2 : 1);
  constexpr int NB = MAXE / RD;  // butterflies per thread per chunk
  const int tid = threadIdx.x, T = blockDim.x;
  const int Ns = 1 << logNs;
  const int logMR = logM - LR, MR = 1 << logMR;
  const int tws = ((1 << logM) >> (logNs + LR)) * twmul;
  for (int t0 = 0; t0 < ntrans; t0 += tpc) {
    const int nt = min(tpc, ntrans - t0);
    const int nb = nt << logMR;
    V v[NB][RD];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int b = tid + i * T;
      if (b < nb) {
        const V* src = buf + (t0 + (b >> logMR)) * stride + (b & (MR - 1));
#pragma unroll
        for (int r = 0; r < RD; ++r) v[i][r] = src[r * MR];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int b = tid + i * T;
      if (b < nb) {
        const int j = b & (MR - 1);
        const int k = j & (Ns - 1);
        V* u = v[i];
        if (Ns > 1) {
          V w1 = tw[k * tws];
          if (INV) w1 = cconj(w1);
          if (RD == 2) {
            u[1] = cmul(u[1], w1);
          } else if (RD == 4) {
            V w2 = tw[2 * k * tws];
            if (INV) w2 = cconj(w2);
            const V w3 = cmul(w1, w2);
            u[1] = cmul(u[1], w1);
            u[2] = cmul(u[2], w2);
            u[3] = cmul(u[3], w3);
          } else {
            V w4 = tw[4 * k * tws];
            if (INV) w4 = cconj(w4);
            const V w2 = cmul(w1, w1), w3 = cmul(w1, w2);
            u[1] = cmul(u[1], w1);
            u[2] = cmul(u[2], w2);
            u[3] = cmul(u[3], w3);
            u[4] = cmul(u[4], w4);
            u[5] = cmul(u[5], cmul(w4, w1));
            u[6] = cmul(u[6], cmul(w4, w2));
            u[7] = cmul(u[7], cmul(w4, w3));
          }
        }
        if (RD == 2) {
          const V a = u[0], c = u[1];
          u[0] = cadd(a, c);
          u[1] = csub(a, c);
        } else if (RD == 4) {
          bfly4<INV>(u[0], u[1], u[2], u[3]);
        } else {
          bfly8<INV>(u);
        }
        V* dst = buf + (t0 + (b >> logMR)) * stride + ((j - k) << LR) + k;
#pragma unroll
        for (int r = 0; r < RD; ++r) dst[r * Ns] = u[r];
      }
    }
    __syncthreads();
  }
}

template <typename real, bool INV, int MAXE>
__device__ void fft_lds(cplx<real>* buf, int M, int ntrans, int stride, const cplx<real>* __restrict__ tw,
                        int twmul) {
  int tpc = (blockDim.x * MAXE) / M;
  if (tpc < 1) tpc = 1;
  const int logM = ilog2(M);
  // Radix-8 passes (stockham_pass<..., 8>) cut the pass count by a third but
  // need ~90 more VGPRs per thread on gfx950, halving occupancy; at the
  // batched sizes that costs more than the saved LDS round trips, so the
  // schedule is radix 4 with one radix-2 pass for odd log2 M.
  for (int logNs = 0; logNs < logM;) {
    const int rem = logM - logNs;
    if (rem >= 2) {
      stockham_pass<real, INV, MAXE, 4>(buf, logM, logNs, ntrans, stride, tw, twmul, tpc);
      logNs += 2;
    } else {
      stockham_pass<real, INV, MAXE, 2>(buf, logM, logNs, ntrans, stride, tw, twmul, tpc);
      logNs += 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Register-resident FFT of length N (power of two) by a group of L = N/E
// lanes holding E elements each: lane l holds x[l + m L], m < E.
// Stockham passes of radix RD (E while the remaining factor allows, then the
// remainder); lane l computes butterflies j = l + t L, t < E/RD.  The inputs
// of butterfly j, x[j + r N/RD], are the lane's own slots v[t + r E/RD] in
// every pass.  Outputs go to the group's LDS area at (j - k) RD + k + s NS
// (k = j mod NS) and are read back in the lane's pattern -- except after
// the last pass, whose outputs j + s N/RD are the lane's own slots.  So a
// forward transform ends, and an inverse one starts, in the load layout: a
// per-mode operator in between needs no data movement, and global loads and
// stores of x[l + m L] are coalesced across lanes.  A group of L <= 64 lanes
// lies in one wavefront, so an exchange is ordered by wave_sync() alone; a
// group of 128 or 256 lanes (1024- and 2048-point columns) spans two or
// four wavefronts of its work-group, which then holds that one group only,
// and an exchange is ordered by a work-group barrier.
// tw holds the (N twmul)-th roots of unity exp(-2 pi i e / (N twmul)); the
// inverse (INV) uses conjugates and is unnormalised.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Barrier of a group of L lanes exchanging through LDS (see above).
template <int L>
__device__ __forceinline__ void group_sync() {
  if constexpr (L <= 64) {
    wave_sync();
  } else {
    __syncthreads();
  }
}

// LDS index of element i of an exchange area (one pad slot per 8 elements,
// so that the stride-RD writes of a pass spread over the banks)
__device__ __forceinline__ int xpad(int i) { return i + (i >> 3); }
template <int N> struct XArea { static constexpr int size = N + N / 8; };

template <bool INV, int RD, typename V>
__device__ __forceinline__ void dft_small(V (&u)[RD]) {
  if constexpr (RD == 2) {
    const V a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  } else if constexpr (RD == 4) {
    bfly4<INV>(u[0], u[1], u[2], u[3]);
  } else {
    bfly8<INV>(u);
  }
}

template <typename real, bool INV, int N, int E, int RD, int NS>
__device__ __forceinline__ void reg_pass(cplx<real> (&v)[E], cplx<real>* x, int lane,
                                         const cplx<real>* __restrict__ tw, int twmul) {
  using V = cplx<real>;
  constexpr int L = N / E, B = E / RD;
  constexpr bool LAST = NS * RD == N;
  constexpr int STEP = N / (NS * RD);
  V o[LAST ? E : 1];
#pragma unroll
  for (int t = 0; t < B; ++t) {
    const int j = lane + t * L;
    const int k = j & (NS - 1);
    V u[RD];
#pragma unroll
    for (int r = 0; r < RD; ++r) u[r] = v[t + r * B];
    if constexpr (NS > 1) {
      const int e = k * STEP * twmul;
      V w1 = tw[e];
      if (INV) w1 = cconj(w1);
      if constexpr (RD == 2) {
        u[1] = cmul(u[1], w1);
      } else {
        V w2 = tw[2 * e];
        if (INV) w2 = cconj(w2);
        const V w3 = cmul(w1, w2);
        u[1] = cmul(u[1], w1);
        u[2] = cmul(u[2], w2);
        u[3] = cmul(u[3], w3);
        if constexpr (RD == 8) {
          V w4 = tw[4 * e];
          if (INV) w4 = cconj(w4);
          u[4] = cmul(u[4], w4);
          u[5] = cmul(u[5], cmul(w4, w1));
          u[6] = cmul(u[6], cmul(w4, w2));
          u[7] = cmul(u[7], cmul(w4, w3));
        }
      }
    }
    dft_small<INV, RD>(u);
    if constexpr (LAST) {
#pragma unroll
      for (int q = 0; q < RD; ++q) o[t + q * B] = u[q];
    } else {
      const int base = (j - k) * RD + k;
#pragma unroll
      for (int q = 0; q < RD; ++q) x[xpad(base + q * NS)] = u[q];
    }
  }
  if constexpr (LAST) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = o[m];
  } else {
    group_sync<L>();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = x[xpad(lane + m * L)];
    group_sync<L>();
  }
}

template <typename real, bool INV, int N, int E, int NS = 1>
__device__ __forceinline__ void reg_fft(cplx<real> (&v)[E], cplx<real>* x, int lane,
                                        const cplx<real>* __restrict__ tw, int twmul) {
  if constexpr (NS < N) {
    // radix E while the remaining factor allows, at most 8 (a lane then
    // computes E / 8 butterflies per pass)
    constexpr int RD0 = (N / NS) >= E ? E : (N / NS);
    constexpr int RD = RD0 > 8 ? 8 : RD0;
    reg_pass<real, INV, N, E, RD, NS>(v, x, lane, tw, twmul);
    reg_fft<real, INV, N, E, NS * RD>(v, x, lane, tw, twmul);
  }
}

// After an M-point complex FFT of z[n] = x[2n] + i x[2n+1] (N = 2M real
// samples), turn Z into the half spectrum of x: bins k = 1..M-1 hold X[k];
// bin 0 holds X[0] + i X[M] (both real).  twN = N-th roots of unity.
template <typename real>
__device__ void r2c_post(cplx<real>* buf, int M, int ntrans, int stride, const cplx<real>* __restrict__ twN) {
  using V = cplx<real>;
  const int half = M >> 1;
  // thread owns bin pair (k, M - k) of every transform; k = 0 packs X[0], X[M]
  for (int t = 0; t < ntrans; ++t) {
    V* z = buf + t * stride;
    for (int k = threadIdx.x; k <= half; k += blockDim.x) {
      if (k == 0) {
        const V z0 = z[0];
        z[0] = mk<V>(z0.x + z0.y, z0.x - z0.y);
      } else {
        const V zk = z[k], zm = z[M - k];
        const V e = cscale(cadd(zk, cconj(zm)), real(0.5));
        const V o = cscale(cmulni(csub(zk, cconj(zm))), real(0.5));
        const V wo = cmul(twN[k], o);
        z[k] = cadd(e, wo);
        z[M - k] = cconj(csub(e, wo));
      }
    }
  }
  __syncthreads();
}

// Inverse of r2c_post: from the packed half spectrum build Z such that the
// unnormalised inverse M-point FFT gives N x[2n] + i N x[2n+1].
template <typename real>
__device__ void c2r_pre(cplx<real>* buf, int M, int ntrans, int stride, const cplx<real>* __restrict__ twN) {
  using V = cplx<real>;
  const int half = M >> 1;
  for (int t = 0; t < ntrans; ++t) {
    V* z = buf + t * stride;
    for (int k = threadIdx.x; k <= half; k += blockDim.x) {
      if (k == 0) {
        const V x0 = z[0];
        z[0] = mk<V>(x0.x + x0.y, x0.x - x0.y);
      } else {
        const V xk = z[k], xm = z[M - k];
        const V a = cadd(xk, cconj(xm));
        const V b = csub(xk, cconj(xm));
        const V iwb = cmuli(cmul(cconj(twN[k]), b));
        z[k] = cadd(a, iwb);
        z[M - k] = cconj(csub(a, iwb));
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions.
// ---------------------------------------------------------------------------
// A wavefront (all 64 lanes active) combines its values in a fixed pattern:
// four DPP steps inside each row of 16 lanes (partner lane i^1, i^2, then the
// mirrored half-row and half of the row), after which every lane of a row
// holds the row's total; the four row totals are then read out and combined
// as (r0 + r1) + (r2 + r3).  Each step adds two values that both partners
// hold, so every lane of a row computes the identical sum; the result is the
// same in every lane and independent of timing.  DPP moves cost a few cycles
// where a cross-lane shuffle through the LDS crossbar costs ~100.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi2, lo2);
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
constexpr int DPP_QUAD_XOR1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int DPP_QUAD_XOR2 = 0x4E;   // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7 - i within 8
constexpr int DPP_ROW_MIRROR = 0x140;   // lane i <-> 15 - i within 16

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<DPP_QUAD_XOR1>(v);
  v += dpp_move<DPP_QUAD_XOR2>(v);
  v += dpp_move<DPP_HALF_MIRROR>(v);
  v += dpp_move<DPP_ROW_MIRROR>(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_move<DPP_QUAD_XOR1>(v));
  v = fmax(v, dpp_move<DPP_QUAD_XOR2>(v));
  v = fmax(v, dpp_move<DPP_HALF_MIRROR>(v));
  v = fmax(v, dpp_move<DPP_ROW_MIRROR>(v));
  return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}

// Reduce NP per-thread accumulators over the block; slot MAXSLOT (if >= 0)
// is reduced with max instead of sum.  Thread 0 writes result i to
// out[i * cstride] (partials are stored component-major, so a wavefront
// reading one component of many work-groups reads contiguous memory).
// red: LDS scratch of at least (blockDim.x/64) * NP doubles.
// Only the first `nused` accumulators (the ones the phase's controller step
// reads) are reduced and stored: each costs a chain of cross-lane steps.
template <int NP>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NP], double* red, double* out, int cstride,
                                                   int nused, int maxslot = -1) {
  if (nused <= 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    if (i < nused) {
      const double v = (i == maxslot) ? wave_max(acc[i]) : wave_sum(acc[i]);
      if (lane == 0) red[wave * NP + i] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      if (i < nused) {
        double s = red[i];
        for (int w = 1; w < nw; ++w) s = (i == maxslot) ? fmax(s, red[w * NP + i]) : s + red[w * NP + i];
        out[(size_t)i * cstride] = s;
      }
    }
  }
}

// Sums (or maxima: bit j of max_mask) of NA arrays of partials, array j
// being p[j][0..cnt[j]), by one wavefront in a fixed order: lane l runs
// through p[j][l], p[j][l + 64], ... in index order, then a butterfly; every
// lane returns the same values.  Used identically by the controller and by
// kernels that need a scalar of the same tick.  The partials are loaded 512
// at a time (eight per lane) for all NA arrays before any of them is summed,
// so the arrays of one controller step cost one memory round trip per 512
// work-groups rather than one per array and per 256.
template <int NA>
__device__ __forceinline__ void wave_reduce_partials_n(const double* const (&p)[NA], const int (&cnt)[NA],
                                                       double (&out)[NA], unsigned max_mask = 0u) {
  const int lane = threadIdx.x & 63;
  double s[NA];
  int cmax = 0;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    s[j] = ((max_mask >> j) & 1u) ? -1.0e300 : 0.0;
    cmax = cnt[j] > cmax ? cnt[j] : cmax;
  }
  for (int base = 0; base < cmax; base += 512) {
    double a[NA][8];
#pragma unroll
    for (int j = 0; j < NA; ++j)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int i = base + lane + 64 * k;
        a[j][k] = i < cnt[j] ? p[j][i] : 0.0;
      }
#pragma unroll
    for (int j = 0; j < NA; ++j)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (base + lane + 64 * k < cnt[j]) s[j] = ((max_mask >> j) & 1u) ? fmax(s[j], a[j][k]) : s[j] + a[j][k];
      }
  }
#pragma unroll
  for (int j = 0; j < NA; ++j) out[j] = ((max_mask >> j) & 1u) ? wave_max(s[j]) : wave_sum(s[j]);
}

__device__ __forceinline__ double wave_reduce_partials(const double* __restrict__ p, int count,
                                                       bool is_max = false) {
  const double* const ps[1] = {p};
  const int cs[1] = {count};
  double o[1];
  wave_reduce_partials_n<1>(ps, cs, o, is_max ? 1u : 0u);
  return o[0];
}

// ---------------------------------------------------------------------------
// Constitutive law in closed form for a 2x2 symmetric strain (xx, yy, xy),
// plane strain (Sec. 2.1).  With m = tr/2, d0 = (exx - eyy)/2,
// r = sqrt(d0^2 + exy^2), eigenvalues e1,2 = m +- r and D = eps - m I, the
// strain-spectral parts are
//   sigma0+- = lam <tr>+- I + mu (s I + q D),
//   s = <e1>+- + <e2>+-,  q = (<e1>+- - <e2>+-) / r,
// evaluated by cases of the signs of e1, e2 so that no 0/0 occurs; in the
// mixed-sign case the D-terms use the unit direction D/r.
// ---------------------------------------------------------------------------
template <typename real>
struct Sym {
  real xx, yy, xy;
};

template <typename real>
__device__ __forceinline__ real ddot(const Sym<real>& a, const Sym<real>& b) {
  return a.xx * b.xx + a.yy * b.yy + real(2) * a.xy * b.xy;
}

// Split part (sign > 0: positive, < 0: negative) of the stress and, if
// `dp` is non-null, its directional derivative along *dp.
template <typename real, int SIGN>
__device__ __forceinline__ void spectral_part(const Sym<real>& e, real lam, real mu, Sym<real>* sig, real* psi,
                                              const Sym<real>* dp, Sym<real>* dsig) {
  const real m = real(0.5) * (e.xx + e.yy);
  const real d0 = real(0.5) * (e.xx - e.yy);
  const real r = sqrt(d0 * d0 + e.xy * e.xy);
  const real e1 = m + r, e2 = m - r;  // e1 >= e2
  const real tr = e.xx + e.yy;
  const bool trpos = SIGN > 0 ? (tr > real(0)) : (tr < real(0));
  const real trp = trpos ? tr : real(0);
  // Cases: both in the part, one (the larger for +, the smaller for -), none.
  const bool both = SIGN > 0 ? (e2 > real(0)) : (e1 < real(0));
  const bool one = SIGN > 0 ? (e1 > real(0)) : (e2 < real(0));
  real s = 0, qd_scale = 0;  // q*D = qd_scale * (D / r) in the mixed case, or 2*D when both
  real ea = 0;               // the eigenvalue in the part (mixed case)
  if (both) {
    s = tr;
  } else if (one) {
    ea = SIGN > 0 ? e1 : e2;
    s = ea;
  }
  if (sig) {
    Sym<real> o;
    const real iso = lam * trp + mu * s;
    if (both) {
      o.xx = iso + real(2) * mu * d0;
      o.yy = iso - real(2) * mu * d0;
      o.xy = real(2) * mu * e.xy;
    } else if (one) {
      // q D = (ea / r) D, |q| <= 2 ; SIGN<0: q = -e2/r
      const real qa = SIGN > 0 ? ea : -ea;  // q * r
      const real ux = d0 / r, uy = e.xy / r;
      o.xx = iso + mu * qa * ux;
      o.yy = iso - mu * qa * ux;
      o.xy = mu * qa * uy;
    } else {
      o.xx = iso;
      o.yy = iso;
      o.xy = 0;
    }
    *sig = o;
  }
  if (psi) {
    real p = real(0.5) * lam * trp * trp;
    if (both)
      p += mu * (e1 * e1 + e2 * e2);
    else if (one)
      p += mu * ea * ea;
    *psi = p;
  }
  if (dp) {
    const Sym<real>& p = *dp;
    const real dtr = p.xx + p.yy, dm = real(0.5) * dtr, dd0 = real(0.5) * (p.xx - p.yy);
    Sym<real> o;
    const real liso = lam * (trpos ? dtr : real(0));
    if (both) {
      o.xx = liso + mu * dtr + real(2) * mu * dd0;
      o.yy = liso + mu * dtr - real(2) * mu * dd0;
      o.xy = real(2) * mu * p.xy;
    } else if (one) {
      const real ux = d0 / r, uy = e.xy / r;
      const real dr = ux * dd0 + uy * p.xy;         // derivative of r
      const real ds = SIGN > 0 ? (dm + dr) : (dm - dr);  // derivative of ea
      // q D = (+-ea) (D/r):  d(qD) = (+-d ea) (D/r) + (+-ea) d(D/r),
      // d(D/r) = (dD - (D/r) dr) / r, dD = (dd0, -dd0, p.xy)
      const real sg = SIGN > 0 ? real(1) : real(-1);
      const real qa = sg * ea;
      const real cr = qa / r;  // in [0, 2]
      const real base = lam * (trpos ? dtr : real(0)) + mu * ds;
      const real t1 = sg * ds - cr * dr;  // coefficient of D/r
      o.xx = base + mu * (t1 * ux + cr * dd0);
      o.yy = base + mu * (-t1 * ux - cr * dd0);
      o.xy = mu * (t1 * uy + cr * p.xy);
    } else {
      o.xx = liso;
      o.yy = liso;
      o.xy = 0;
    }
    *dsig = o;
  }
}

// Volumetric-deviatoric split (plane strain, zero out-of-plane strain):
//   psi0+ = K <tr>+^2 / 2 + mu (eps:eps - tr^2 / 3),  psi0- = K <tr>-^2 / 2,
//   sigma0+ = (K <tr>+ - 2 mu tr / 3) I + 2 mu eps,   sigma0- = K <tr>- I,
// K = lam + 2 mu / 3; the tangent differentiates the ramps with [tr > 0],
// [tr < 0].
template <typename real>
__device__ __forceinline__ Sym<real> voldev_stress(const Sym<real>& e, real lam, real mu, real hk) {
  const real K = lam + real(2) * mu / real(3);
  const real tr = e.xx + e.yy;
  const real tp = tr > real(0) ? tr : real(0), tm = tr < real(0) ? tr : real(0);
  const real iso = hk * (K * tp - real(2) * mu * tr / real(3)) + K * tm;
  Sym<real> o;
  o.xx = iso + hk * real(2) * mu * e.xx;
  o.yy = iso + hk * real(2) * mu * e.yy;
  o.xy = hk * real(2) * mu * e.xy;
  return o;
}
template <typename real>
__device__ __forceinline__ Sym<real> voldev_tangent(const Sym<real>& e, const Sym<real>& p, real lam, real mu,
                                                    real hk) {
  const real K = lam + real(2) * mu / real(3);
  const real tr = e.xx + e.yy, dtr = p.xx + p.yy;
  const real vol = (tr > real(0) ? hk * K : real(0)) + (tr < real(0) ? K : real(0));
  const real iso = vol * dtr - hk * real(2) * mu * dtr / real(3);
  Sym<real> o;
  o.xx = iso + hk * real(2) * mu * p.xx;
  o.yy = iso + hk * real(2) * mu * p.yy;
  o.xy = hk * real(2) * mu * p.xy;
  return o;
}

// Full stress sigma = hk sigma0+ + sigma0-, hk = h(phi) + k_res.
template <typename real>
__device__ __forceinline__ Sym<real> stress(const Sym<real>& e, real lam, real mu, real hk, int split) {
  Sym<real> o;
  if (split == 2) return voldev_stress(e, lam, mu, hk);
  if (split == 0) {
    const real tr = e.xx + e.yy;
    o.xx = hk * (lam * tr + real(2) * mu * e.xx);
    o.yy = hk * (lam * tr + real(2) * mu * e.yy);
    o.xy = hk * (real(2) * mu * e.xy);
    return o;
  }
  Sym<real> sp, sm;
  spectral_part<real, +1>(e, lam, mu, &sp, nullptr, nullptr, nullptr);
  spectral_part<real, -1>(e, lam, mu, &sm, nullptr, nullptr, nullptr);
  o.xx = hk * sp.xx + sm.xx;
  o.yy = hk * sp.yy + sm.yy;
  o.xy = hk * sp.xy + sm.xy;
  return o;
}

// Tangent action C : p at strain e.
template <typename real>
__device__ __forceinline__ Sym<real> tangent(const Sym<real>& e, const Sym<real>& p, real lam, real mu, real hk,
                                             int split) {
  Sym<real> o;
  if (split == 2) return voldev_tangent(e, p, lam, mu, hk);
  if (split == 0) {
    const real tr = p.xx + p.yy;
    o.xx = hk * (lam * tr + real(2) * mu * p.xx);
    o.yy = hk * (lam * tr + real(2) * mu * p.yy);
    o.xy = hk * (real(2) * mu * p.xy);
    return o;
  }
  Sym<real> dp, dm;
  spectral_part<real, +1>(e, lam, mu, nullptr, nullptr, &p, &dp);
  spectral_part<real, -1>(e, lam, mu, nullptr, nullptr, &p, &dm);
  o.xx = hk * dp.xx + dm.xx;
  o.yy = hk * dp.yy + dm.yy;
  o.xy = hk * dp.xy + dm.xy;
  return o;
}

// psi0+ and psi0- (isotropic model: psi0+ = full energy, psi0- = 0).
template <typename real>
__device__ __forceinline__ void energies(const Sym<real>& e, real lam, real mu, int split, real* pp, real* pm) {
  if (split == 2) {
    const real K = lam + real(2) * mu / real(3);
    const real tr = e.xx + e.yy;
    const real tp = tr > real(0) ? tr : real(0), tm = tr < real(0) ? tr : real(0);
    *pp = real(0.5) * K * tp * tp + mu * (e.xx * e.xx + e.yy * e.yy + real(2) * e.xy * e.xy - tr * tr / real(3));
    *pm = real(0.5) * K * tm * tm;
    return;
  }
  if (split == 0) {
    const real tr = e.xx + e.yy;
    *pp = real(0.5) * lam * tr * tr + mu * (e.xx * e.xx + e.yy * e.yy + real(2) * e.xy * e.xy);
    *pm = 0;
    return;
  }
  spectral_part<real, +1>(e, lam, mu, nullptr, pp, nullptr, nullptr);
  spectral_part<real, -1>(e, lam, mu, nullptr, pm, nullptr, nullptr);
}

}  // namespace spff
