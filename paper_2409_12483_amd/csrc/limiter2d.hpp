// Kernels of the limited 2-D step: a posteriori subcell ADER-WENO2 limiting
// of the 2-D ADER-DG step (Sec. 1.4 and Sec. 1.6 with d = 2), compiled as
// part of dg2d.hip (they share its operator and WENO tables).  The candidate
// is the DG step of dg2d.hip on a mesh padded with one ghost cell per side
// (periodic images, or mirror images for free outflow); then, per step:
//   detect    PAD on the candidate's nodes and (P (x) P) subcell averages, NAD
//             against the extrema of v^n over the cell and its eight vertex
//             neighbours (delta = max(1e-4, 1e-3 (max - min)) per variable);
//   subgrid   for a troubled cell, one ADER-WENO2 step (WENO of degree 1 along
//             x then y, the degree-1 space-time predictor, Rusanov fluxes) of
//             its N_s x N_s subcells from v^n, with the DG step's dt, one
//             workgroup per cell and one thread per subcell of the cell and
//             its ring of neighbouring subcells;
//   subgrid0  when that left the admissible set in any troubled cell, the
//             first-order redo (Rusanov fluxes of the averages) of every
//             troubled cell;
//   finish    u = (R (x) R) v for a troubled cell, scaled toward its mean
//             until admissible; for an unlimited cell the candidate, with the
//             flux of every face it shares with a troubled cell replaced, per
//             face node k, by sum_s F_s (integral of phi_k over sub-face s) /
//             (N_s w_k); v^{n+1}; the signal speed of the final state; the
//             status E_NONPHYS when a subcell average of v^{n+1} is not
//             admissible.
// The exchange changes unlimited cells after their detection, so subgrid,
// subgrid0 and finish run in up to three passes (the detection / correction
// cascade): an unlimited cell whose corrected state fails PAD is marked with
// the next pass's number and recomputed like the others; troubled[c] holds
// the pass in which a cell was found troubled (1 = by the detectors).  The
// passes write uout / vout; the last one also writes the step's result back.
#pragma once

#include "launch_lim.hpp"

namespace aderdg {

__constant__ DevLimR c2_limR[kDevMaxn];

hipError_t upload_lim2d_tables(const void* limR) {
  return hipMemcpyToSymbol(HIP_SYMBOL(c2_limR), limR, sizeof(DevLimR) * kDevMaxn);
}

// Interior cell of index i in [-1, C] along one axis: itself, its periodic
// image, or (free outflow) the boundary cell whose mirror image it is.
__device__ __forceinline__ int64_t lim2_src(int64_t i, int64_t C, int bc, bool& mir) {
  mir = false;
  if (i >= 0 && i < C) return i;
  if (bc == kLim2Periodic) return i < 0 ? i + C : i - C;
  mir = true;
  return i < 0 ? 0 : C - 1;
}

// ------------------------------------------------------- copies, ghosts ----
__global__ void __launch_bounds__(256) lim2d_copy_kernel(Lim2Args L, int to_padded, int per_cell) {
  const int64_t total = L.cx * L.cy * per_cell;
  const int64_t py = L.cy + 2;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t c = e / per_cell, k = e - c * per_cell;
    const int64_t ix = c / L.cy, iy = c - ix * L.cy;
    const int64_t p = ((ix + 1) * py + iy + 1) * per_cell + k;
    if (to_padded) L.up[p] = L.u[e];
    else L.u[e] = L.up[p];
  }
}

template <int N>
__global__ void __launch_bounds__(256) lim2d_ghost_kernel(Lim2Args L) {
  constexpr int n = N + 1, LL = n * n, M = 4;
  const int64_t px = L.cx + 2, py = L.cy + 2;
  const int64_t nghost = 2 * py + 2 * L.cx;
  const int64_t total = nghost * LL * M;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t g = e / (LL * M);
    const int k = (int)(e - g * (LL * M)), node = k / M, r = k - node * M;
    int64_t gx, gy;                                   // padded coordinates of ghost g
    if (g < py) { gx = 0; gy = g; }
    else if (g < 2 * py) { gx = px - 1; gy = g - py; }
    else if (g < 2 * py + L.cx) { gx = g - 2 * py + 1; gy = 0; }
    else { gx = g - 2 * py - L.cx + 1; gy = py - 1; }
    bool mx, my;
    const int64_t sx = lim2_src(gx - 1, L.cx, L.bc, mx), sy = lim2_src(gy - 1, L.cy, L.bc, my);
    const int i = node / n, j = node - i * n;
    const int si = mx ? n - 1 - i : i, sj = my ? n - 1 - j : j;
    L.up[((gx * py + gy) * LL + node) * M + r] = L.up[(((sx + 1) * py + sy + 1) * LL + si * n + sj) * M + r];
  }
}

// v = (P (x) P) u of every interior cell, from the caller's state.
template <int N>
__global__ void __launch_bounds__(256) lim2d_project_kernel(Lim2Args L) {
  constexpr int n = N + 1, LL = n * n, M = 4, Ns = 2 * N + 1;
  __shared__ double U[LL * M];
  __shared__ double V1[Ns * n * M];
  const int64_t c = blockIdx.x;
  for (int k = threadIdx.x; k < LL * M; k += 256) U[k] = L.u[c * LL * M + k];
  __syncthreads();
  for (int w = threadIdx.x; w < Ns * n * M; w += 256) {
    const int s = w / (n * M), j = (w / M) % n, r = w % M;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc = fma(c2_ops[N].P[s][i], U[(i * n + j) * M + r], acc);
    V1[w] = acc;
  }
  __syncthreads();
  for (int w = threadIdx.x; w < Ns * Ns * M; w += 256) {
    const int s = w / (Ns * M), t = (w / M) % Ns, r = w % M;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc = fma(c2_ops[N].P[t][j], V1[(s * n + j) * M + r], acc);
    L.v[c * Ns * Ns * M + w] = acc;
  }
}

// Subcell averages (P (x) P) X of one cell's nodal values X [n][n][4] (LDS)
// into S [Ns][Ns][4] (LDS), through the x-projected T [Ns][n][4].
template <int N>
__device__ __forceinline__ void lim2_project(const double* X, double* T, double* S) {
  constexpr int n = N + 1, M = 4, Ns = 2 * N + 1;
  for (int w = threadIdx.x; w < Ns * n * M; w += blockDim.x) {
    const int s = w / (n * M), j = (w / M) % n, r = w % M;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc = fma(c2_ops[N].P[s][i], X[(i * n + j) * M + r], acc);
    T[w] = acc;
  }
  __syncthreads();
  for (int w = threadIdx.x; w < Ns * Ns * M; w += blockDim.x) {
    const int s = w / (Ns * M), t = (w / M) % Ns, r = w % M;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc = fma(c2_ops[N].P[t][j], T[(s * n + j) * M + r], acc);
    S[w] = acc;
  }
  __syncthreads();
}

// ------------------------------------------------------------- detect ----
template <int N>
__global__ void __launch_bounds__(256) lim2d_detect_kernel(Lim2Args L) {
  constexpr int n = N + 1, LL = n * n, M = 4, Ns = 2 * N + 1, S2 = Ns * Ns;
  __shared__ double X[LL * M], T[Ns * n * M], S[S2 * M];
  __shared__ double bc2[2];
  __shared__ double ext[8][8];                        // per wave: min[4], max[4]
  double t;
  const double dt = step_dt2d<N>(L.dg, t, bc2, false);
  if (!(dt > 0.0)) return;
  const int64_t c = blockIdx.x, ix = c / L.cy, iy = c - ix * L.cy;
  const int64_t py = L.cy + 2;
  if (c == 0 && threadIdx.x == 0) L.cnt[2] = 0ull;    // the redo flag of this step
  const double* cand = L.up + ((ix + 1) * py + iy + 1) * LL * M;
  for (int k = threadIdx.x; k < LL * M; k += 256) X[k] = cand[k];
  // extrema of v^n over the cell and its eight vertex neighbours
  double mn[M], mx[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    mn[r] = INFINITY;
    mx[r] = -INFINITY;
  }
  for (int w = threadIdx.x; w < 9 * S2; w += 256) {
    const int nb = w / S2, sub = w - nb * S2;
    bool m1, m2;
    const int64_t sx = lim2_src(ix + nb / 3 - 1, L.cx, L.bc, m1), sy = lim2_src(iy + nb % 3 - 1, L.cy, L.bc, m2);
    const double* vv = L.v + ((sx * L.cy + sy) * S2 + sub) * M;
#pragma unroll
    for (int r = 0; r < M; ++r) {
      mn[r] = fmin(mn[r], vv[r]);
      mx[r] = fmax(mx[r], vv[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < M; ++r) {
    for (int off = 32; off > 0; off >>= 1) {
      mn[r] = fmin(mn[r], __shfl_xor(mn[r], off, 64));
      mx[r] = fmax(mx[r], __shfl_xor(mx[r], off, 64));
    }
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int r = 0; r < M; ++r) {
      ext[wv][r] = mn[r];
      ext[wv][4 + r] = mx[r];
    }
  }
  __syncthreads();
  lim2_project<N>(X, T, S);                           // ends with a barrier
  double lo[M], hi[M];
#pragma unroll
  for (int r = 0; r < M; ++r) {
    double a = ext[0][r], b = ext[0][4 + r];
    for (int w = 1; w < 4; ++w) {
      a = fmin(a, ext[w][r]);
      b = fmax(b, ext[w][4 + r]);
    }
    const double delta = fmax(1.0e-4, 1.0e-3 * (b - a));
    lo[r] = a - delta;
    hi[r] = b + delta;
  }
  bool bad = false;
  for (int w = threadIdx.x; w < S2; w += 256) {
    const double* q = S + w * M;
#pragma unroll
    for (int r = 0; r < M; ++r) bad |= !(q[r] >= lo[r] && q[r] <= hi[r]);
    bad |= !Euler2::admissible(q, L.dg.gamma);
  }
  for (int w = threadIdx.x; w < LL; w += 256) bad |= !Euler2::admissible(X + w * M, L.dg.gamma);
  const bool any = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    L.troubled[c] = any ? 1 : 0;
    if (any) atomicAdd(&L.cnt[0], 1ull);
  }
}

// ------------------------------------------------------------ subgrid ----
// Geometry: the averages of a troubled cell's subcells and two rings around
// them (E x E, E = Ns + 4) in LDS; threads over the cell's subcells and one
// ring (H x H, H = Ns + 2), which are reconstructed and predicted; the faces
// of the cell's subcells take the Rusanov fluxes of the predicted traces.
template <int N>
struct Sub2Geo {
  static constexpr int Ns = 2 * N + 1, E = Ns + 4, H = Ns + 2, M = 4;
  static constexpr int NT = ((H * H + 63) / 64) * 64;
  static constexpr int VA = E * E * M, WX = H * E * 2 * M, TRX = H * H * 2 * 2 * 2 * M;
  static constexpr int BUF = (VA + WX > TRX ? VA + WX : TRX);
};

// Rusanov flux of the subgrid along DIR, integrated over the face's two time
// and two face nodes (weights of the degree-1 rule), scaled by sc.
template <int DIR>
__device__ __forceinline__ void sub_face_flux(const double* tm, const double* tp, double sc, double gamma,
                                              double* F) {
#pragma unroll
  for (int r = 0; r < 4; ++r) F[r] = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      double G[4];
      rusanov2<DIR>(tm + (a * 2 + k) * 4, tp + (a * 2 + k) * 4, G, gamma);
      const double wk = c2_ops[1].w[a] * c2_ops[1].w[k];
#pragma unroll
      for (int r = 0; r < 4; ++r) F[r] = fma(wk, sc * G[r], F[r]);
    }
}

template <int N>
__global__ void __launch_bounds__(Sub2Geo<N>::NT) lim2d_subgrid_kernel(Lim2Args L) {
  using G = Sub2Geo<N>;
  constexpr int Ns = G::Ns, E = G::E, H = G::H, M = 4;
  __shared__ double buf[G::BUF];
  __shared__ double bc2[2];
  double* const va = buf;                     // [E][E][M]
  double* const wx = buf + G::VA;             // [H (x)][E (y)][2 (x node)][M]
  double* const trx = buf;                    // [H][H][2 faces][2 time][2 nodes][M] (after the sweeps)
  const int64_t c = blockIdx.x;
  // found troubled in this pass (uniform per workgroup); checked before the
  // step size, whose read and barrier would otherwise cost every idle workgroup
  if (L.troubled[c] != L.pass + 1) return;
  double t;
  const double dt = step_dt2d<N>(L.dg, t, bc2, false);
  if (!(dt > 0.0)) return;
  const int64_t ix = c / L.cy, iy = c - ix * L.cy;
  const double gamma = L.dg.gamma, gm1 = gamma - 1.0;
  const double dxs = L.dg.dx / Ns, dys = L.dg.dy / Ns;
  const DevWeno& WT = c2_weno[0];
  // averages of the E x E tile: subgrid index ix Ns - 2 + X along x
  for (int e = threadIdx.x; e < E * E; e += G::NT) {
    const int X = e / E, Y = e - X * E;
    const int64_t gx = ix * Ns - 2 + X, gy = iy * Ns - 2 + Y;
    const int64_t cxg = gx < 0 ? -1 : gx / Ns, cyg = gy < 0 ? -1 : gy / Ns;
    int sx = (int)(gx - cxg * Ns), sy = (int)(gy - cyg * Ns);
    bool m1, m2;
    const int64_t ox = lim2_src(cxg, L.cx, L.bc, m1), oy = lim2_src(cyg, L.cy, L.bc, m2);
    if (m1) sx = Ns - 1 - sx;
    if (m2) sy = Ns - 1 - sy;
    const double* src = L.v + (((ox * L.cy + oy) * Ns + sx) * Ns + sy) * M;
#pragma unroll
    for (int r = 0; r < M; ++r) va[e * M + r] = src[r];
  }
  __syncthreads();
  // WENO along x at the two x nodes, for columns 1..H of the tile and every row
  for (int e = threadIdx.x; e < H * E * M; e += G::NT) {
    const int hx = e / (E * M), Y = (e / M) % E, r = e % M;
    double row[3], o[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) row[d] = va[((hx + d) * E + Y) * M + r];
    weno1d<1>(row, WT, o, -1);
    wx[((hx * E + Y) * 2 + 0) * M + r] = o[0];
    wx[((hx * E + Y) * 2 + 1) * M + r] = o[1];
  }
  __syncthreads();
  // this thread's subcell of the H x H region: (hx, hy), tile column hx + 1
  const int tid = threadIdx.x;
  const bool live = tid < H * H;
  const int hx = live ? tid / H : 0, hy = live ? tid - (tid / H) * H : 0;
  double w[2][2][M];                          // nodal WENO values [x node][y node][r]
#pragma unroll
  for (int kx = 0; kx < 2; ++kx)
#pragma unroll
    for (int r = 0; r < M; ++r) {
      double col[3], o[2];
#pragma unroll
      for (int d = 0; d < 3; ++d) col[d] = wx[((hx * E + hy + d) * 2 + kx) * M + r];
      weno1d<1>(col, WT, o, -1);
      w[kx][0][r] = o[0];
      w[kx][1][r] = o[1];
    }
  // degree-1 space-time predictor of the subcell (Picard, the subcell's own stopping test)
  double q[2][2][2][M];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < M; ++r) q[a][i][j][r] = w[i][j][r];
  const double cx_ = dt / dxs, cy_ = dt / dys, tol = L.dg.tol;
  for (int it = 0; it < L.dg.max_iter; ++it) {
    double fx[2][2][2][M], fy[2][2][2][M];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          Euler2::flux_x(q[a][i][j], fx[a][i][j], gm1);
          Euler2::flux_y(q[a][i][j], fy[a][i][j], gm1);
        }
    double e = 0.0, qm = 0.0;
    double qn[2][2][2][M];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < M; ++r) {
          double kf[2];
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            double sx = 0.0, sy = 0.0;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
              sx += c2_ops[1].ktil[i][p] * (cx_ * fx[b][p][j][r]);
              sy += c2_ops[1].ktil[j][p] * (cy_ * fy[b][i][p][r]);
            }
            kf[b] = -(sx + sy);
          }
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            const double v = w[i][j][r] + (c2_ops[1].kappa[a][0] * kf[0] + c2_ops[1].kappa[a][1] * kf[1]);
            e = fmax(e, fabs(v - q[a][i][j][r]));
            qm = fmax(qm, fabs(v));
            qn[a][i][j][r] = v;
          }
        }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < M; ++r) q[a][i][j][r] = qn[a][i][j][r];
    if (e <= tol * fmax(1.0, qm)) break;
  }
  // face traces of the subcell: x faces [W, E][a][node along y], y faces [S, N][a][node along x]
  double tw[2][2][M], te[2][2][M], ts[2][2][M], tn[2][2][M];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int r = 0; r < M; ++r) {
        tw[a][k][r] = c2_ops[1].psi0[0] * q[a][0][k][r] + c2_ops[1].psi0[1] * q[a][1][k][r];
        te[a][k][r] = c2_ops[1].psi1[0] * q[a][0][k][r] + c2_ops[1].psi1[1] * q[a][1][k][r];
        ts[a][k][r] = c2_ops[1].psi0[0] * q[a][k][0][r] + c2_ops[1].psi0[1] * q[a][k][1][r];
        tn[a][k][r] = c2_ops[1].psi1[0] * q[a][k][0][r] + c2_ops[1].psi1[1] * q[a][k][1][r];
      }
  __syncthreads();                            // the tile and the x sweep are dead from here
  constexpr int TS = 2 * 2 * 2 * M;           // doubles per subcell: 2 faces x 2 time x 2 nodes x M
  if (live) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int r = 0; r < M; ++r) {
          trx[tid * TS + ((0 * 2 + a) * 2 + k) * M + r] = tw[a][k][r];
          trx[tid * TS + ((1 * 2 + a) * 2 + k) * M + r] = te[a][k][r];
        }
  }
  __syncthreads();
  // x faces of the cell's subcells: the thread of subcell (hx, hy), 1 <= hx, hy <= Ns
  const bool own = live && hx >= 1 && hx <= Ns && hy >= 1 && hy <= Ns;
  double FW[M], FE[M], FS[M], FN[M];
  if (own) {
    const double* mine = trx + tid * TS;
    sub_face_flux<0>(trx + (tid - H) * TS + 1 * 2 * 2 * M, mine + 0, cx_, gamma, FW);   // west face
    sub_face_flux<0>(mine + 1 * 2 * 2 * M, trx + (tid + H) * TS + 0, cx_, gamma, FE);    // east face
  }
  __syncthreads();
  if (live) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int r = 0; r < M; ++r) {
          trx[tid * TS + ((0 * 2 + a) * 2 + k) * M + r] = ts[a][k][r];
          trx[tid * TS + ((1 * 2 + a) * 2 + k) * M + r] = tn[a][k][r];
        }
  }
  __syncthreads();
  if (own) {
    const double* mine = trx + tid * TS;
    sub_face_flux<1>(trx + (tid - 1) * TS + 1 * 2 * 2 * M, mine + 0, cy_, gamma, FS);    // south face
    sub_face_flux<1>(mine + 1 * 2 * 2 * M, trx + (tid + 1) * TS + 0, cy_, gamma, FN);    // north face
    const int s = hx - 1, tt = hy - 1;
    double vn[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      const double v0 = L.v[(((c * Ns + s) * Ns) + tt) * M + r];
      vn[r] = v0 - (FE[r] - FW[r]) - (FN[r] - FS[r]);
      L.vfv[(((c * Ns + s) * Ns) + tt) * M + r] = vn[r];
    }
    double* sf = L.sflux + c * 4 * Ns * M;
#pragma unroll
    for (int r = 0; r < M; ++r) {
      if (s == 0) sf[(0 * Ns + tt) * M + r] = FW[r];
      if (s == Ns - 1) sf[(1 * Ns + tt) * M + r] = FE[r];
      if (tt == 0) sf[(2 * Ns + s) * M + r] = FS[r];
      if (tt == Ns - 1) sf[(3 * Ns + s) * M + r] = FN[r];
    }
    if (!Euler2::admissible(vn, gamma)) atomicCAS(&L.cnt[2], 0ull, (unsigned long long)(L.pass + 1));
  }
}

// First-order redo of every troubled cell (Rusanov fluxes of the subcell
// averages), when the ADER-WENO2 subgrid step left the admissible set.
template <int N>
__global__ void __launch_bounds__(256) lim2d_subgrid0_kernel(Lim2Args L) {
  constexpr int Ns = 2 * N + 1, M = 4;
  __shared__ double bc2[2];
  if (!L.cnt[2]) return;                       // no redo this step (checked before the step size)
  const int64_t c = blockIdx.x;
  const int tv = L.troubled[c];
  if (tv < 1 || tv > L.pass + 1) return;
  double t;
  const double dt = step_dt2d<N>(L.dg, t, bc2, false);
  if (!(dt > 0.0)) return;
  const int64_t ix = c / L.cy, iy = c - ix * L.cy;
  const double gamma = L.dg.gamma;
  const double cx_ = dt / (L.dg.dx / Ns), cy_ = dt / (L.dg.dy / Ns);
  auto avg = [&](int64_t gx, int64_t gy, double* o) {
    const int64_t cxg = gx < 0 ? -1 : gx / Ns, cyg = gy < 0 ? -1 : gy / Ns;
    int sx = (int)(gx - cxg * Ns), sy = (int)(gy - cyg * Ns);
    bool m1, m2;
    const int64_t ox = lim2_src(cxg, L.cx, L.bc, m1), oy = lim2_src(cyg, L.cy, L.bc, m2);
    if (m1) sx = Ns - 1 - sx;
    if (m2) sy = Ns - 1 - sy;
    const double* src = L.v + (((ox * L.cy + oy) * Ns + sx) * Ns + sy) * M;
#pragma unroll
    for (int r = 0; r < M; ++r) o[r] = src[r];
  };
  for (int w = threadIdx.x; w < Ns * Ns; w += 256) {
    const int s = w / Ns, tt = w - s * Ns;
    const int64_t gx = ix * Ns + s, gy = iy * Ns + tt;
    double q0[M], qw[M], qe[M], qs[M], qn[M], FW[M], FE[M], FS[M], FN[M];
    avg(gx, gy, q0);
    avg(gx - 1, gy, qw);
    avg(gx + 1, gy, qe);
    avg(gx, gy - 1, qs);
    avg(gx, gy + 1, qn);
    rusanov2<0>(qw, q0, FW, gamma);
    rusanov2<0>(q0, qe, FE, gamma);
    rusanov2<1>(qs, q0, FS, gamma);
    rusanov2<1>(q0, qn, FN, gamma);
    double* sf = L.sflux + c * 4 * Ns * M;
#pragma unroll
    for (int r = 0; r < M; ++r) {
      FW[r] *= cx_;
      FE[r] *= cx_;
      FS[r] *= cy_;
      FN[r] *= cy_;
      L.vfv[(((c * Ns + s) * Ns) + tt) * M + r] = q0[r] - (FE[r] - FW[r]) - (FN[r] - FS[r]);
      if (s == 0) sf[(0 * Ns + tt) * M + r] = FW[r];
      if (s == Ns - 1) sf[(1 * Ns + tt) * M + r] = FE[r];
      if (tt == 0) sf[(2 * Ns + s) * M + r] = FS[r];
      if (tt == Ns - 1) sf[(3 * Ns + s) * M + r] = FN[r];
    }
  }
}

// ------------------------------------------------------------- finish ----
// Whether pass L.pass can change cell c's result: it or a face neighbour was
// found troubled in the previous pass, or the first-order redo began in this
// pass.
__device__ __forceinline__ bool lim2_changed(const Lim2Args& L, int64_t c) {
  const int64_t ix = c / L.cy, iy = c - ix * L.cy;
  bool changed = L.troubled[c] == L.pass + 1 || L.cnt[2] == (unsigned long long)(L.pass + 1);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int64_t jx = ix + (f == 0 ? -1 : f == 1 ? 1 : 0), jy = iy + (f == 2 ? -1 : f == 3 ? 1 : 0);
    const bool inside = (jx >= 0 && jx < L.cx && jy >= 0 && jy < L.cy);
    bool m1, m2;
    const int64_t o = lim2_src(jx, L.cx, L.bc, m1) * L.cy + lim2_src(jy, L.cy, L.bc, m2);
    changed |= (inside || L.bc == kLim2Periodic) && L.troubled[o] == L.pass + 1;
  }
  return changed;
}

template <int N>
__global__ void __launch_bounds__(256) lim2d_finish_kernel(Lim2Args L) {
  constexpr int n = N + 1, LL = n * n, M = 4, Ns = 2 * N + 1, S2 = Ns * Ns;
  __shared__ double U[Corr2Geo<N>::CPB * LL * M], V1[Corr2Geo<N>::CPB * Ns * n * M];
  __shared__ double Ub[LL * M], S[S2 * M], T[Ns * n * M];
  __shared__ double dG[4][n * M];
  __shared__ double part[8], bc2[2], mean[M];
  __shared__ int okf;
  const int64_t c = blockIdx.x, ix = c / L.cy, iy = c - ix * L.cy;
  // a middle pass leaves an unchanged cell alone; decided before the step size,
  // whose read and barrier would otherwise cost every idle workgroup
  if (L.pass > 0 && L.pass < L.npass - 1 && !lim2_changed(L, c)) return;
  double t;
  const double dt = step_dt2d<N>(L.dg, t, bc2, false);
  if (!(dt > 0.0)) return;
  const int64_t py = L.cy + 2;
  const double* const up = L.up + ((ix + 1) * py + iy + 1) * LL * M;    // the candidate
  double* const uo = L.uout + c * LL * M;
  double* const vc = L.vout + c * S2 * M;
  const bool last = L.pass == L.npass - 1;
  const int tv = L.troubled[c];
  const bool bad = tv >= 1 && tv <= L.pass + 1;       // uniform per workgroup
  if (last && c == 0 && threadIdx.x == 0) {
    if (L.cnt[2]) atomicAdd(&L.cnt[1], 1ull);
  }
  // a later pass recomputes a cell only if it or a face neighbour was found
  // troubled in the previous pass, or the first-order redo began in this pass
  bool keep = false;
  if (L.pass > 0 && !lim2_changed(L, c)) {
    keep = true;                                       // last pass: the previous pass's result stands
    for (int w = threadIdx.x; w < LL * M; w += 256) U[w] = uo[w];
  }
  if (keep) {
  } else if (bad) {
    // u = (R (x) R) v through the x-reconstructed [n][Ns][M] (in S's place: T is [Ns][n])
    const double* vf = L.vfv + c * S2 * M;
    for (int k = threadIdx.x; k < S2 * M; k += 256) S[k] = vf[k];
    __syncthreads();
    if (threadIdx.x < M) {
      double m = 0.0;
      for (int k = 0; k < S2; ++k) m += S[k * M + threadIdx.x];
      mean[threadIdx.x] = m / S2;
    }
    for (int w = threadIdx.x; w < n * Ns * M; w += 256) {
      const int i = w / (Ns * M), tt = (w / M) % Ns, r = w % M;
      double acc = 0.0;
      for (int s = 0; s < Ns; ++s) acc = fma(c2_limR[N].R[i][s], S[(s * Ns + tt) * M + r], acc);
      T[w] = acc;                                     // [i][tt][r]
    }
    __syncthreads();
    for (int w = threadIdx.x; w < LL * M; w += 256) {
      const int i = w / (n * M), j = (w / M) % n, r = w % M;
      double acc = 0.0;
      for (int tt = 0; tt < Ns; ++tt) acc = fma(c2_limR[N].R[j][tt], T[(i * Ns + tt) * M + r], acc);
      U[w] = acc;                                     // R v
    }
    __syncthreads();
    // the largest theta in {1, 1/2, ..., 2^-11} with u and (P (x) P) u admissible, else the mean
    double theta = 1.0;
    bool done = false;
    for (int k = 0; k < 12 && !done; ++k) {
      for (int w = threadIdx.x; w < LL * M; w += 256) Ub[w] = mean[w % M] + theta * (U[w] - mean[w % M]);
      __syncthreads();
      lim2_project<N>(Ub, T, S);
      bool ok = true;
      for (int w = threadIdx.x; w < S2; w += 256) ok &= Euler2::admissible(S + w * M, L.dg.gamma);
      for (int w = threadIdx.x; w < LL; w += 256) ok &= Euler2::admissible(Ub + w * M, L.dg.gamma);
      done = __syncthreads_and(ok);
      theta *= 0.5;
    }
    if (!done) {
      for (int w = threadIdx.x; w < LL * M; w += 256) Ub[w] = mean[w % M];
    }
    __syncthreads();
    for (int w = threadIdx.x; w < LL * M; w += 256) uo[w] = Ub[w];
    for (int k = threadIdx.x; k < S2 * M; k += 256) vc[k] = vf[k];
    for (int w = threadIdx.x; w < LL * M; w += 256) U[w] = Ub[w];
  } else {
    // the candidate; the faces shared with troubled cells take the subgrid flux
    for (int w = threadIdx.x; w < LL * M; w += 256) Ub[w] = up[w];
    // face f: 0 west, 1 east, 2 south, 3 north
    bool nbad[4];
    int64_t nb[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int64_t jx = ix + (f == 0 ? -1 : f == 1 ? 1 : 0), jy = iy + (f == 2 ? -1 : f == 3 ? 1 : 0);
      const bool inside = (jx >= 0 && jx < L.cx && jy >= 0 && jy < L.cy);
      bool m1, m2;
      nb[f] = lim2_src(jx, L.cx, L.bc, m1) * L.cy + lim2_src(jy, L.cy, L.bc, m2);
      const int tn = (inside || L.bc == kLim2Periodic) ? L.troubled[nb[f]] : 0;
      nbad[f] = tn >= 1 && tn <= L.pass + 1;        // a mark of this pass (racing write) counts next pass
    }
    for (int w = threadIdx.x; w < 4 * n * M; w += 256) {
      const int f = w / (n * M), k = (w / M) % n, r = w % M;
      double d = 0.0;
      if (nbad[f]) {
        // the neighbour's face on this side: W <-> E, S <-> N
        const int of = f ^ 1;
        const double* Fs = L.sflux + (nb[f] * 4 + of) * Ns * M;
        double acc = 0.0;
        for (int s = 0; s < Ns; ++s) acc = fma(c2_ops[N].P[s][k], Fs[s * M + r], acc);
        const double Gp = acc / (double(Ns) * double(Ns) * c2_ops[N].w[k]);
        // the DG flux of that face: the east (north) face flux of the padded cell on its minus side
        const int64_t gx = ix + 1 - (f == 0 ? 1 : 0), gy = iy + 1 - (f == 2 ? 1 : 0);
        const double Gd = L.dg.gface[(((gx * py + gy) * 2 + (f >> 1)) * n + k) * M + r];
        d = Gp - Gd;
      }
      dG[f][k * M + r] = d;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < LL * M; w += 256) {
      const int i = w / (n * M), j = (w / M) % n, r = w % M;
      double val = Ub[w];
      if (nbad[0]) val += c2_ops[N].psi0[i] * c2_ops[N].winv[i] * dG[0][j * M + r];
      if (nbad[1]) val -= c2_ops[N].psi1[i] * c2_ops[N].winv[i] * dG[1][j * M + r];
      if (nbad[2]) val += c2_ops[N].psi0[j] * c2_ops[N].winv[j] * dG[2][i * M + r];
      if (nbad[3]) val -= c2_ops[N].psi1[j] * c2_ops[N].winv[j] * dG[3][i * M + r];
      U[w] = val;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < LL * M; w += 256) uo[w] = U[w];
    lim2_project<N>(U, T, S);
    for (int k = threadIdx.x; k < S2 * M; k += 256) vc[k] = S[k];
    if (!last) {
      // the cascade: a corrected state that fails PAD joins the troubled cells
      bool fail = false;
      for (int w = threadIdx.x; w < S2; w += 256) fail |= !Euler2::admissible(S + w * M, L.dg.gamma);
      for (int w = threadIdx.x; w < LL; w += 256) fail |= !Euler2::admissible(U + w * M, L.dg.gamma);
      if (__syncthreads_or(fail) && threadIdx.x == 0) {
        L.troubled[c] = L.pass + 2;
        atomicAdd(&L.cnt[0], 1ull);
      }
    }
  }
  if (!last) return;                                  // uniform: signal speeds and status of the final pass
  __syncthreads();
  // status: the subcell averages v^{n+1} (the data the detectors and the
  // subgrid scheme start from) must be admissible; a polynomial may dip below
  // zero at a node between them, and its next candidate then fails PAD
  bool badu = false;
  for (int w = threadIdx.x; w < S2; w += 256) badu |= !Euler2::admissible(vc + w * M, L.dg.gamma);
  if (__any(badu) && (threadIdx.x & 63) == 0)
    atomicMin(&L.dg.clk->stat[(blockIdx.x + (threadIdx.x >> 6)) % kSlots].v, -5);
  // the step's result: the state into the padded state's interior (this cell's
  // candidate is no longer read), the subcell averages into v (read by no
  // kernel of this pass)
  double* const upw = L.up + ((ix + 1) * py + iy + 1) * LL * M;
  for (int w = threadIdx.x; w < LL * M; w += 256) upw[w] = U[w];
  for (int k = threadIdx.x; k < S2 * M; k += 256) L.v[c * S2 * M + k] = vc[k];
  double lx, ly;
  subcell_speeds<N>(U, V1, 1, L.dg.gamma, lx, ly);
  publish_lambda(*L.dg.clk, (L.dg.step + 1) % 3, lx, ly, part);
}

// ----------------------------------------------------------- launchers ----
#define ADERDG_LIM2_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9)

hipError_t launch_lim2d_copy(const Lim2Args& L, int to_padded, hipStream_t st) {
  const int n = L.N + 1, per_cell = n * n * 4;
  int64_t blocks = (L.cx * L.cy * per_cell + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(lim2d_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, L, to_padded, per_cell);
  return hipGetLastError();
}

hipError_t launch_lim2d_ghosts(const Lim2Args& L, hipStream_t st) {
  const int n = L.N + 1;
  int64_t blocks = ((2 * (L.cy + 2) + 2 * L.cx) * n * n * 4 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  switch (L.N) {
#define X(NN) case NN: hipLaunchKernelGGL((lim2d_ghost_kernel<NN>), dim3((unsigned)blocks), dim3(256), 0, st, L); break;
    ADERDG_LIM2_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lim2d_project(const Lim2Args& L, hipStream_t st) {
  const dim3 grid((unsigned)(L.cx * L.cy));
  switch (L.N) {
#define X(NN) case NN: hipLaunchKernelGGL((lim2d_project_kernel<NN>), grid, dim3(256), 0, st, L); break;
    ADERDG_LIM2_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N>
static hipError_t lim2_after(const Lim2Args& L0, hipStream_t st) {
  const dim3 grid((unsigned)(L0.cx * L0.cy));
  hipLaunchKernelGGL((lim2d_detect_kernel<N>), grid, dim3(256), 0, st, L0);
  hipError_t e = hipGetLastError();
  for (int p = 0; p < L0.npass && e == hipSuccess; ++p) {
    Lim2Args L = L0;
    L.pass = p;
    hipLaunchKernelGGL((lim2d_subgrid_kernel<N>), grid, dim3(Sub2Geo<N>::NT), 0, st, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((lim2d_subgrid0_kernel<N>), grid, dim3(256), 0, st, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((lim2d_finish_kernel<N>), grid, dim3(256), 0, st, L);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_lim2d_after_candidate(const Lim2Args& L, hipStream_t st) {
  switch (L.N) {
#define X(NN) case NN: return lim2_after<NN>(L, st);
    ADERDG_LIM2_CASES(X)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace aderdg
