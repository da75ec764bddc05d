// Downstream helix fit of the track candidates (the step that consumes the
// chain's output, Section 2.2.2: candidates are lists of spacepoints whose track
// parameters are fitted next).  For a solenoid field B along z, per candidate
// (a label carried by at least min_hits spacepoints):
//   transverse plane: the algebraic circle fit, the least-squares solution of
//     X^2 + Y^2 + D X + E Y + F = 0, centre (-D/2, -E/2), R^2 = D^2/4 + E^2/4 - F,
//     solved from its normal equations in coordinates centred on the hits' mean
//     (the fit is translation invariant; centring keeps the FP64 system well
//     conditioned); pT = 0.3 B R, charge from the turning sense of the
//     innermost-to-outermost chord about the centre, phi0 = the direction of
//     motion at the point of closest approach to the origin;
//   longitudinal: least-squares line z = z0 + s tan(lambda) over the arc length
//     s = 2 R asin(rho / 2R), eta = asinh(tan(lambda)).
// Hits are grouped by label with a stable least-significant-digit radix sort of
// the hit ids keyed by label (8-bit digits), so that each candidate's hits come in
// ascending id order, and each wave sums its candidate's moments in a fixed order:
// the results do not depend on scheduling, and the sort costs the same for a giant
// candidate as for many small ones.
#include <math.h>

#include "../../include/trk.h"
#include "common.h"
#include "ctx.h"
#include "kernels.h"

namespace {

__global__ void label_count(const int* __restrict__ labels, int n, int* cnt, int* d_err) {
  GRID_STRIDE(i, n) {
    const int l = labels[i];
    if ((unsigned)l < (unsigned)n) atomicAdd(&cnt[l], 1);
    else atomicOr(d_err, TRK_ERRBIT_INDEX);
  }
}

__global__ void label_flags(const int* __restrict__ cnt, int n, int min_hits, int* flag) {
  GRID_STRIDE(l, n) flag[l] = cnt[l] >= min_hits ? 1 : 0;
}

// Radix pass, step 1: count of each digit (key >> shift) & 255 in every chunk of
// FIT_SORT_CHUNK keys, stored digit-major (hist[d * nb + chunk]) so that one
// exclusive scan gives every (digit, chunk) its first output position.
constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = FIT_SORT_CHUNK / RS_THREADS;

__global__ __launch_bounds__(RS_THREADS) void radix_hist(const int* __restrict__ keys, int n, int shift, int nb,
                                                         int* __restrict__ hist) {
  __shared__ int cnt[256];
  const int t = threadIdx.x;
  cnt[t] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * FIT_SORT_CHUNK;
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t e = base + r * RS_THREADS + t;
    if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(size_t)t * nb + blockIdx.x] = cnt[t];
}

// Radix pass, step 2: stable scatter.  The chunk is taken in rounds of 256 keys in
// index order; an element's place among the equal digits of its round is its rank
// in its wave's match group (eight ballots) plus the counts of the same digit in the
// round's earlier waves, after the counts of the chunk's earlier rounds.
// vin == nullptr: the values are the indices themselves.
__global__ __launch_bounds__(RS_THREADS) void radix_scatter(const int* __restrict__ kin, const int* __restrict__ vin,
                                                            int n, int shift, int nb, const int* __restrict__ off,
                                                            int* __restrict__ kout, int* __restrict__ vout) {
  constexpr int NWV = RS_THREADS / 64;
  __shared__ int base[256], running[256], wc[NWV][256];
  const int t = threadIdx.x, w = t >> 6, l = lane_id();
  base[t] = off[(size_t)t * nb + blockIdx.x];
  running[t] = 0;
  const unsigned long long below = l == 0 ? 0ull : (~0ull >> (64 - l));
  for (int r = 0; r < RS_ROUNDS; ++r) {
#pragma unroll
    for (int q = 0; q < NWV; ++q) wc[q][t] = 0;
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * FIT_SORT_CHUNK + r * RS_THREADS + t;
    const bool valid = e < n;
    const int k = valid ? kin[e] : 0;
    const int v = valid ? (vin ? vin[e] : (int)e) : 0;
    const int d = (k >> shift) & 255;
    unsigned long long m = ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const unsigned long long bb = ballot(bit);
      m &= bit ? bb : ~bb;
    }
    // the highest lane of a match group records the group's size
    if (valid && (m >> l) == 1ull) wc[w][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      int pos = base[d] + running[d] + __popcll(m & below);
      for (int q = 0; q < w; ++q) pos += wc[q][d];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int q = 0; q < NWV; ++q) add += wc[q][t];
    running[t] += add;
  }
}

// candidate c (in label order) -> its label and hit count
__global__ void cand_list(const int* __restrict__ cnt, const int* __restrict__ cidx, int n, int min_hits,
                          int64_t cap, int* cand_label, int* cand_nhits) {
  GRID_STRIDE(l, n) {
    if (cnt[l] >= min_hits) {
      const int c = cidx[l];
      if (c < cap) {
        cand_label[c] = (int)l;
        cand_nhits[c] = cnt[l];
      }
    }
  }
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct HitXY {
  double X, Y, Z, rho;
};

__device__ __forceinline__ HitXY hit_at(const float* __restrict__ x, int h) {
  const double rho = 1000.0 * (double)x[3 * (size_t)h];
  const double phi = M_PI * (double)x[3 * (size_t)h + 1];
  HitXY p;
  p.X = rho * cos(phi);
  p.Y = rho * sin(phi);
  p.Z = 1000.0 * (double)x[3 * (size_t)h + 2];
  p.rho = rho;
  return p;
}

// one wave per candidate; params[c] = (pT, phi0, eta, z0, q, chi2_xy)
__global__ __launch_bounds__(256) void helix_fit_kernel(const float* __restrict__ x, const int* __restrict__ hits,
                                                        const int* __restrict__ start, const int* __restrict__ cand_label,
                                                        const int* __restrict__ cand_nhits, const int* d_ncand,
                                                        int64_t cap, double b_field, double* __restrict__ params) {
  const int l = lane_id();
  const int64_t nc = min((int64_t)*d_ncand, cap);
  const int waves = gridDim.x * (blockDim.x >> 6);
  for (int64_t c = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < nc; c += waves) {
    const int lab = cand_label[c], nh = cand_nhits[c];
    const int* hl = hits + start[lab];
    const double inv_n = 1.0 / (double)nh;
    // pass 1: the mean position
    double sx = 0.0, sy = 0.0;
    for (int k = l; k < nh; k += 64) {
      const HitXY p = hit_at(x, hl[k]);
      sx += p.X;
      sy += p.Y;
    }
    const double mx = wsum(sx) * inv_n, my = wsum(sy) * inv_n;
    // pass 2: moments of the centred coordinates; innermost and outermost hits
    double m_xx = 0, m_xy = 0, m_yy = 0, m_x = 0, m_y = 0, m_xr = 0, m_yr = 0, m_r = 0;
    double rmin = INFINITY, rmax = -INFINITY;
    int imin = 0x7fffffff, imax = 0x7fffffff;   // hit ids of the extreme rho (smallest id on ties)
    for (int k = l; k < nh; k += 64) {
      const int h = hl[k];
      const HitXY p = hit_at(x, h);
      const double u = p.X - mx, v = p.Y - my, r2 = u * u + v * v;
      m_xx += u * u; m_xy += u * v; m_yy += v * v; m_x += u; m_y += v;
      m_xr += u * r2; m_yr += v * r2; m_r += r2;
      if (p.rho < rmin || (p.rho == rmin && h < imin)) { rmin = p.rho; imin = h; }
      if (p.rho > rmax || (p.rho == rmax && h < imax)) { rmax = p.rho; imax = h; }
    }
    m_xx = wsum(m_xx); m_xy = wsum(m_xy); m_yy = wsum(m_yy); m_x = wsum(m_x); m_y = wsum(m_y);
    m_xr = wsum(m_xr); m_yr = wsum(m_yr); m_r = wsum(m_r);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double r1 = __shfl_xor(rmin, o, 64), r2 = __shfl_xor(rmax, o, 64);
      const int i1 = __shfl_xor(imin, o, 64), i2 = __shfl_xor(imax, o, 64);
      if (r1 < rmin || (r1 == rmin && i1 < imin)) { rmin = r1; imin = i1; }
      if (r2 > rmax || (r2 == rmax && i2 < imax)) { rmax = r2; imax = i2; }
    }
    // normal equations [m_xx m_xy m_x; m_xy m_yy m_y; m_x m_y n] [D E F] = -[m_xr m_yr m_r]
    const double a11 = m_xx, a12 = m_xy, a13 = m_x, a22 = m_yy, a23 = m_y, a33 = (double)nh;
    const double b1 = -m_xr, b2 = -m_yr, b3 = -m_r;
    const double c11 = a22 * a33 - a23 * a23, c12 = a13 * a23 - a12 * a33, c13 = a12 * a23 - a13 * a22;
    const double det = a11 * c11 + a12 * c12 + a13 * c13;
    const double c22 = a11 * a33 - a13 * a13, c23 = a12 * a13 - a11 * a23, c33 = a11 * a22 - a12 * a12;
    // collinear or coincident transverse positions: no circle (NaN parameters)
    const bool degenerate = !(fabs(det) > 1e-13 * fabs(a11 * a22 * a33));
    const double D = (c11 * b1 + c12 * b2 + c13 * b3) / det;
    const double E = (c12 * b1 + c22 * b2 + c23 * b3) / det;
    const double Fc = (c13 * b1 + c23 * b2 + c33 * b3) / det;
    const double cu = -0.5 * D, cv = -0.5 * E;            // centre in centred coordinates
    const double R = sqrt(fmax(cu * cu + cv * cv - Fc, 0.0));
    const double a = cu + mx, b = cv + my;                 // centre
    // pass 3: arc lengths, the line z(s) and the transverse residuals
    double ss = 0, sss = 0, sz = 0, ssz = 0, chi = 0;
    for (int k = l; k < nh; k += 64) {
      const HitXY p = hit_at(x, hl[k]);
      const double s = R > 0.0 ? 2.0 * R * asin(fmin(1.0, p.rho / (2.0 * R))) : p.rho;
      ss += s; sss += s * s; sz += p.Z; ssz += s * p.Z;
      const double d = hypot(p.X - a, p.Y - b) - R;
      chi += d * d;
    }
    ss = wsum(ss); sss = wsum(sss); sz = wsum(sz); ssz = wsum(ssz); chi = wsum(chi);
    if (l == 0) {
      const double tl = ((double)nh * ssz - ss * sz) / ((double)nh * sss - ss * ss);
      const double z0 = (sz - tl * ss) * inv_n;
      const HitXY pn = hit_at(x, imin), pf = hit_at(x, imax);
      const double cross = (pf.X - pn.X) * (b - pn.Y) - (pf.Y - pn.Y) * (a - pn.X);
      const double q = cross < 0.0 ? 1.0 : -1.0;
      double phi0 = atan2(b, a) + q * M_PI / 2.0;
      phi0 = phi0 - 2.0 * M_PI * floor((phi0 + M_PI) / (2.0 * M_PI));
      double* o = params + 6 * c;
      if (degenerate) {
        for (int k = 0; k < 6; ++k) o[k] = NAN;
        continue;
      }
      o[0] = 0.3 * b_field * R / 1000.0;
      o[1] = phi0;
      o[2] = asinh(tl);
      o[3] = z0;
      o[4] = q;
      o[5] = chi * inv_n;
    }
  }
}

}  // namespace

extern "C" int trk_fit(trk_ctx* c, const float* d_x, int64_t n, const int32_t* d_labels, int32_t min_hits,
                       double b_field, int32_t* d_cand_label, int32_t* d_cand_nhits, double* d_params, int64_t cap,
                       int64_t* n_cands, hipStream_t s) {
  if (!c || n < 0 || n > c->cfg.max_hits || min_hits < 1 || cap < 0 || !n_cands) return TRK_E_INVAL;
  CtxStreamScope scope(c, s);
  if (n > 0 && (!d_x || !d_labels)) return TRK_E_INVAL;
  if (cap > 0 && (!d_cand_label || !d_cand_nhits || !d_params)) return TRK_E_INVAL;
  *n_cands = 0;
  if (hipSetDevice(c->device) != hipSuccess) return TRK_E_DEVICE;
  if (n == 0) return TRK_OK;
  const int nn = (int)n;
  int* err = &c->dev_words[0];
  int* d_total = &c->dev_words[4];
  launch_fill_int(err, 0, 1, s);
  launch_fill_int(c->fit_cnt, 0, nn + 1, s);
  label_count<<<blocks_for(nn, 256), 256, 0, s>>>(d_labels, nn, c->fit_cnt, err);
  label_flags<<<blocks_for(nn, 256), 256, 0, s>>>(c->fit_cnt, nn, min_hits, c->fit_flag);
  launch_scan_excl(c->fit_flag, c->fit_cidx, nn, nullptr, d_total, c->graph.tmp, s);
  launch_scan_excl(c->fit_cnt, c->fit_start, nn, nullptr, nullptr, c->graph.tmp, s);
  // hit ids ordered by (label, id): passes over the digits of keys < n, the last
  // pass writing into fit_hits
  {
    int bits = 1;
    while (bits < 31 && (1 << bits) < nn) ++bits;
    const int passes = (bits + 7) / 8;
    const int nb = (int)fit_sort_blocks(nn);
    int* kbuf[2] = {c->fit_keys, c->fit_keys2};
    int* vbuf[2] = {c->fit_raw, c->fit_hits};
    const int* kin = d_labels;
    const int* vin = nullptr;
    for (int p = 0; p < passes; ++p) {
      const int o = (passes - 1 - p) % 2 == 0 ? 1 : 0;
      radix_hist<<<nb, RS_THREADS, 0, s>>>(kin, nn, 8 * p, nb, c->fit_hist);
      launch_scan_excl(c->fit_hist, c->fit_hoff, (int64_t)256 * nb, nullptr, nullptr, c->graph.tmp, s);
      radix_scatter<<<nb, RS_THREADS, 0, s>>>(kin, vin, nn, 8 * p, nb, c->fit_hoff, kbuf[o], vbuf[o]);
      kin = kbuf[o];
      vin = vbuf[o];
    }
  }
  if (cap > 0) {
    cand_list<<<blocks_for(nn, 256), 256, 0, s>>>(c->fit_cnt, c->fit_cidx, nn, min_hits, cap, d_cand_label,
                                                   d_cand_nhits);
    helix_fit_kernel<<<c->n_cu * 4, 256, 0, s>>>(d_x, c->fit_hits, c->fit_start, d_cand_label, d_cand_nhits, d_total,
                                                  cap, b_field, d_params);
  }
  int words[5] = {0, 0, 0, 0, 0};
  if (hipMemcpyAsync(words, c->dev_words, sizeof(words), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess)
    return TRK_E_DEVICE;
  if (words[0]) return TRK_E_INVAL;
  *n_cands = words[4];
  return words[4] > cap ? TRK_E_CAPACITY : TRK_OK;
}
