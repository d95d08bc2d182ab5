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
// held in LDS, transform t at buf + t*stride.  Radix-4 passes, one radix-2
// pass when log2 M is odd.  Pass with sub-transform size Ns and radix Rd:
//   j in [0, M/Rd), k = j mod Ns
//   v_r = x[j + r M/Rd] * w_{Ns Rd}^{r k}          (twiddle)
//   v'  = DFT_Rd(v)
//   y[(j - k) Rd + k + s Ns] = v'_s
// Each pass reads its inputs into registers, synchronises, then writes in
// place (chunks of whole transforms, at most T*MAXE elements per chunk).
// tw holds the (M*twmul)-th roots of unity exp(-2 pi i e/(M twmul)); the
// inverse transform (INV) uses their conjugates and is unnormalised.
// Requires M <= blockDim.x * MAXE.
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

template <typename real, bool INV, int MAXE>
__device__ void fft_lds(cplx<real>* buf, int M, int ntrans, int stride, const cplx<real>* __restrict__ tw,
                        int twmul) {
  using V = cplx<real>;
  const int tid = threadIdx.x, T = blockDim.x;
  int tpc = (T * MAXE) / M;
  if (tpc < 1) tpc = 1;
  const int logM = ilog2(M);
  for (int logNs = 0; logNs < logM;) {
    const int Ns = 1 << logNs;
    const bool r4 = (logM - logNs) >= 2;
    if (r4) {
      const int logMR = logM - 2, MR = 1 << logMR;
      const int tws = (M >> (logNs + 2)) * twmul;
      for (int t0 = 0; t0 < ntrans; t0 += tpc) {
        const int nt = min(tpc, ntrans - t0);
        const int nb = nt << logMR;
        V v[MAXE];
#pragma unroll
        for (int i = 0; i < MAXE / 4; ++i) {
          const int b = tid + i * T;
          if (b < nb) {
            const int t = t0 + (b >> logMR), j = b & (MR - 1);
            const V* src = buf + t * stride + j;
            v[4 * i + 0] = src[0];
            v[4 * i + 1] = src[MR];
            v[4 * i + 2] = src[2 * MR];
            v[4 * i + 3] = src[3 * MR];
          }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXE / 4; ++i) {
          const int b = tid + i * T;
          if (b < nb) {
            const int t = t0 + (b >> logMR), j = b & (MR - 1);
            const int k = j & (Ns - 1);
            V v0 = v[4 * i], v1 = v[4 * i + 1], v2 = v[4 * i + 2], v3 = v[4 * i + 3];
            if (Ns > 1) {
              V w1 = tw[k * tws], w2 = tw[2 * k * tws], w3 = tw[3 * k * tws];
              if (INV) {
                w1 = cconj(w1);
                w2 = cconj(w2);
                w3 = cconj(w3);
              }
              v1 = cmul(v1, w1);
              v2 = cmul(v2, w2);
              v3 = cmul(v3, w3);
            }
            bfly4<INV>(v0, v1, v2, v3);
            V* dst = buf + t * stride + ((j - k) << 2) + k;
            dst[0] = v0;
            dst[Ns] = v1;
            dst[2 * Ns] = v2;
            dst[3 * Ns] = v3;
          }
        }
        __syncthreads();
      }
      logNs += 2;
    } else {
      const int logMR = logM - 1, MR = 1 << logMR;
      const int tws = (M >> (logNs + 1)) * twmul;
      for (int t0 = 0; t0 < ntrans; t0 += tpc) {
        const int nt = min(tpc, ntrans - t0);
        const int nb = nt << logMR;
        V v[MAXE];
#pragma unroll
        for (int i = 0; i < MAXE / 2; ++i) {
          const int b = tid + i * T;
          if (b < nb) {
            const int t = t0 + (b >> logMR), j = b & (MR - 1);
            const V* src = buf + t * stride + j;
            v[2 * i + 0] = src[0];
            v[2 * i + 1] = src[MR];
          }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXE / 2; ++i) {
          const int b = tid + i * T;
          if (b < nb) {
            const int t = t0 + (b >> logMR), j = b & (MR - 1);
            const int k = j & (Ns - 1);
            V v0 = v[2 * i], v1 = v[2 * i + 1];
            if (Ns > 1) {
              V w1 = tw[k * tws];
              if (INV) w1 = cconj(w1);
              v1 = cmul(v1, w1);
            }
            V* dst = buf + t * stride + ((j - k) << 1) + k;
            dst[0] = cadd(v0, v1);
            dst[Ns] = csub(v0, v1);
          }
        }
        __syncthreads();
      }
      logNs += 1;
    }
  }
}

// After an M-point complex FFT of z[n] = x[2n] + i x[2n+1] (N = 2M real
// samples), turn Z into the half spectrum of x: bins k = 1..M-1 hold X[k];
// bin 0 holds X[0] + i X[M] (both real).  twN = N-th roots of unity.
template <typename real>
__device__ void r2c_post(cplx<real>* buf, int M, int ntrans, int stride, const cplx<real>* __restrict__ twN) {
  using V = cplx<real>;
  const int half = M >> 1, per = half + 1;
  const int total = ntrans * per;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int t = idx / per, k = idx - t * per;
    V* z = buf + t * stride;
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
  __syncthreads();
}

// Inverse of r2c_post: from the packed half spectrum build Z such that the
// unnormalised inverse M-point FFT gives N x[2n] + i N x[2n+1].
template <typename real>
__device__ void c2r_pre(cplx<real>* buf, int M, int ntrans, int stride, const cplx<real>* __restrict__ twN) {
  using V = cplx<real>;
  const int half = M >> 1, per = half + 1;
  const int total = ntrans * per;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int t = idx / per, k = idx - t * per;
    V* z = buf + t * stride;
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
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Reduce NP per-thread accumulators over the block; slot MAXSLOT (if >= 0)
// is reduced with max instead of sum.  Thread 0 writes the NP results to out.
// red: LDS scratch of at least (blockDim.x/64) * NP doubles.
template <int NP>
__device__ void block_reduce_store(double (&acc)[NP], double* red, double* out, int maxslot = -1) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const double v = (i == maxslot) ? wave_max(acc[i]) : wave_sum(acc[i]);
    if (lane == 0) red[wave * NP + i] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double s = red[i];
      for (int w = 1; w < nw; ++w) s = (i == maxslot) ? fmax(s, red[w * NP + i]) : s + red[w * NP + i];
      out[i] = s;
    }
  }
}

// Sum (or max) of `count` partials p[i*stride] by one wavefront in a fixed
// order; every lane returns the same value.  Used identically by the
// controller and by kernels that need a scalar of the same tick.
__device__ __forceinline__ double wave_reduce_partials(const double* __restrict__ p, int count, int stride,
                                                       bool is_max = false) {
  const int lane = threadIdx.x & 63;
  double s = is_max ? -1.0e300 : 0.0;
  for (int i = lane; i < count; i += 64) s = is_max ? fmax(s, p[i * stride]) : s + p[i * stride];
  return is_max ? wave_max(s) : wave_sum(s);
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

// Full stress sigma = hk sigma0+ + sigma0-, hk = h(phi) + k_res.
template <typename real>
__device__ __forceinline__ Sym<real> stress(const Sym<real>& e, real lam, real mu, real hk, int split) {
  Sym<real> o;
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
