// Surface loads of the heartbeat test (Sec. 4): a follower pressure on the
// endocardium and elastic Robin springs on the epicardium.
//
// Each face node sums the contributions of its incident faces (P1 faces: eight
// lanes per node, each taking every eighth face, summed by a fixed butterfly;
// 6-node faces: one thread per node, in increasing face order) and writes the
// node's three values to a dense per-dof buffer (zero off the face nodes); the
// element kernels add that buffer when they finalize each node.  No atomics:
// the result is bitwise reproducible.
//
// Pressure p (times the load scale) on a flat triangle with current vertices
// x0, x1, x2 (outward from the body): each vertex gets p (x1-x0) x (x2-x0) / 6
// in the residual, and p [(v1-v0) x (x2-x0) + (x1-x0) x (v2-v0)] / 6 in the
// Jacobian action (not symmetric).  Springs with reference unit normal N and
// area A: the residual gains M K u with M_ab = A (1 + delta_ab) / 12 and
// K = k_par I + (k_perp - k_par) N (x) N (symmetric, constant).  A follower
// traction t (fixed direction, per unit current area, times the load scale
// s) gives each vertex s t l / 6 with l = |(x1-x0) x (x2-x0)|, subtracted
// from the residual; in the Jacobian action s t (n . dl_v) / 6 with
// dl_v = (v1-v0) x (x2-x0) + (x1-x0) x (v2-v0), n = the unit normal; its own
// 3x3 block at vertex a is -s/6 t (x) dl/dx_a, dl/dx_0 = (e1 - e2) x n,
// dl/dx_1 = e2 x n, dl/dx_2 = n x e1 (e1 = x1 - x0, e2 = x2 - x0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "nle_internal.hpp"

namespace nle {

namespace {

template <typename T>
struct SurfArgs {
  int64_t nsn;
  int32_t npf, ntf;
  const int32_t *node, *ptr, *ent, *tri;
  const uint32_t *fmask;  // per face: Dirichlet bits of vertex a at bits 3a..3a+2
  const T *pgeo, *rgeo;
  double p;             // effective pressure (residual)
  double s;             // load scale (residual, diagonal)
  const double *plin;   // effective pressure and load scale at the linearization (Jacobian action)
  double tf[3];         // follower traction
  double kperp, kpar;
  int32_t damp;         // dashpots: velocity vt + cv (u - ut) through cperp, cpar
  double cperp, cpar, cv;
  const double *vt, *ut;
  const T *u, *v;
  T *fs;
  double *red;          // energy partials (one per workgroup)
  const int32_t *skip;
  int32_t nomask;       // Jv: keep v on Dirichlet dofs
};

template <typename T>
__device__ __forceinline__ void cross_acc(const T a[3], const T b[3], T s, T acc[3]) {
  acc[0] += s * (a[1] * b[2] - a[2] * b[1]);
  acc[1] += s * (a[2] * b[0] - a[0] * b[2]);
  acc[2] += s * (a[0] * b[1] - a[1] * b[0]);
}

// Contributions of face f to node g (a vertex of f), added to acc.
template <typename T, int OP>
__device__ __forceinline__ void surface_face(const SurfArgs<T> &A, int32_t g, int32_t f, T pe,
                                             T acc[3]) {
  const int32_t n[3] = {A.tri[3 * f], A.tri[3 * f + 1], A.tri[3 * f + 2]};
  if (f < A.npf + A.ntf) {
    const bool trac = f >= A.npf;
    if (OP == OP_RES || OP == OP_JV || (trac && (OP == OP_DIAG || OP == OP_ODIAG))) {
      const T *Xf = A.pgeo + 9 * int64_t(f);
      T x[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) x[a][i] = Xf[3 * a + i] + A.u[3 * int64_t(n[a]) + i];
      T e1[3], e2[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        e1[i] = x[1][i] - x[0][i];
        e2[i] = x[2][i] - x[0][i];
      }
      const T s = pe / T(6);
      if (trac) {
        T a2[3] = {T(0), T(0), T(0)};
        cross_acc(e1, e2, T(1), a2);
        const T l = sqrt(a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]);
        const T tv[3] = {T(A.tf[0]), T(A.tf[1]), T(A.tf[2])};
        // the Jacobian action and the (lazily formed) nodal blocks use the
        // load scale of the linearization
        const T sc = ((OP == OP_JV || OP == OP_ODIAG) ? T(A.plin[1]) : T(A.s)) / T(6);
        if (OP == OP_RES) {
#pragma unroll
          for (int i = 0; i < 3; ++i) acc[i] -= sc * l * tv[i];
        } else if (OP == OP_JV) {
          const uint32_t fm = A.nomask ? 0u : A.fmask[f];
          T d1[3], d2[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            const T v0 = ((fm >> i) & 1u) ? T(0) : A.v[3 * int64_t(n[0]) + i];
            const T v1 = ((fm >> (3 + i)) & 1u) ? T(0) : A.v[3 * int64_t(n[1]) + i];
            const T v2 = ((fm >> (6 + i)) & 1u) ? T(0) : A.v[3 * int64_t(n[2]) + i];
            d1[i] = v1 - v0;
            d2[i] = v2 - v0;
          }
          T da[3] = {T(0), T(0), T(0)};
          cross_acc(d1, e2, T(1), da);
          cross_acc(e1, d2, T(1), da);
          const T dl = (a2[0] * da[0] + a2[1] * da[1] + a2[2] * da[2]) / l;
#pragma unroll
          for (int i = 0; i < 3; ++i) acc[i] -= sc * dl * tv[i];
        } else {
          // this node's own block: -s/6 t (x) dl/dx_a
          const int a = n[0] == g ? 0 : (n[1] == g ? 1 : 2);
          const T nh[3] = {a2[0] / l, a2[1] / l, a2[2] / l};
          T w[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) w[i] = a == 0 ? e1[i] - e2[i] : (a == 1 ? e2[i] : T(0));
          T ga[3] = {T(0), T(0), T(0)};
          if (a == 2)
            cross_acc(nh, e1, T(1), ga);
          else
            cross_acc(w, nh, T(1), ga);
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            if (OP == OP_DIAG)
              acc[i] -= sc * tv[i] * ga[i];
            else
              acc[i] -= T(0.5) * sc * (tv[i] * ga[(i + 1) % 3] + ga[i] * tv[(i + 1) % 3]);
          }
        }
      } else if (OP == OP_RES) {
        cross_acc(e1, e2, s, acc);
      } else if (OP == OP_JV) {
        // the tangent has identity rows and columns on Dirichlet dofs:
        // v's prescribed components do not enter the coupling
        const uint32_t fm = A.nomask ? 0u : A.fmask[f];
        T d1[3], d2[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const T v0 = ((fm >> i) & 1u) ? T(0) : A.v[3 * int64_t(n[0]) + i];
          const T v1 = ((fm >> (3 + i)) & 1u) ? T(0) : A.v[3 * int64_t(n[1]) + i];
          const T v2 = ((fm >> (6 + i)) & 1u) ? T(0) : A.v[3 * int64_t(n[2]) + i];
          d1[i] = v1 - v0;
          d2[i] = v2 - v0;
        }
        cross_acc(d1, e2, s, acc);
        cross_acc(e1, d2, s, acc);
      }
    }
  } else {
    const T *R = A.rgeo + 4 * int64_t(f - A.npf - A.ntf);
    const T N[3] = {R[0], R[1], R[2]};
    const T area = R[3];
    const T kpar = T(A.kpar), dk = T(A.kperp - A.kpar);
    // the dashpots' force C (vt + cv (u - ut)) adds cv C to the tangent
    const T kpe = A.damp ? T(A.kpar + A.cv * A.cpar) : kpar;
    const T dke = A.damp ? T(A.kperp - A.kpar + A.cv * (A.cperp - A.cpar)) : dk;
    if (OP == OP_DIAG) {
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] += area / T(6) * (kpe + dke * N[i] * N[i]);
    } else if (OP == OP_ODIAG) {
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] += area / T(6) * dke * N[i] * N[(i + 1) % 3];
    } else {
      const T *w = OP == OP_JV ? A.v : A.u;
      const uint32_t fm = (OP == OP_JV && !A.nomask) ? A.fmask[f] : 0u;
      const T kw = OP == OP_JV ? kpe : kpar, dw = OP == OP_JV ? dke : dk;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const T m = area / T(12) * (n[b] == g ? T(2) : T(1));
        const int64_t nb = int64_t(n[b]);
        T wb[3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
          wb[i] = ((fm >> (3 * b + i)) & 1u) ? T(0) : w[3 * nb + i];
        const T nw = N[0] * wb[0] + N[1] * wb[1] + N[2] * wb[2];
#pragma unroll
        for (int i = 0; i < 3; ++i) acc[i] += m * (kw * wb[i] + dw * nw * N[i]);
        if (OP == OP_RES && A.damp) {
          T z[3];
#pragma unroll
          for (int i = 0; i < 3; ++i)
            z[i] = T(A.vt[3 * nb + i] + A.cv * (double(A.u[3 * nb + i]) - A.ut[3 * nb + i]));
          const T nz = N[0] * z[0] + N[1] * z[1] + N[2] * z[2];
          const T cpar = T(A.cpar), dc = T(A.cperp - A.cpar);
#pragma unroll
          for (int i = 0; i < 3; ++i) acc[i] += m * (cpar * z[i] + dc * nz * N[i]);
        }
      }
    }
  }
}

// SL lanes per face node: lane j of a node takes its incident faces j, j + SL,
// ... (in increasing face order) and the node's lanes, which are consecutive
// and aligned in a wave, are summed by a fixed butterfly.  SL = 8 keeps a face
// node's ~6 dependent face loads in flight together; the energy (one partial
// per workgroup of nodes) runs with SL = 1.
template <typename T, int OP, int SL>
__global__ __launch_bounds__(NT) void k_surface(SurfArgs<T> A) {
  __shared__ double sh[NT / 64];
  if (A.skip && A.skip[0] != 0) return;
  const int64_t t = int64_t(blockIdx.x) * NT + threadIdx.x;
  const int64_t k = t / SL;
  const int sub = int(t % SL);
  double e = 0.0;
  T acc[3] = {T(0), T(0), T(0)};
  int32_t g = 0;
  if (k < A.nsn) {
    g = A.node[k];
    const T pe = OP == OP_JV ? T(A.plin[0]) : T(A.p);
    for (int q = A.ptr[k] + sub; q < A.ptr[k + 1]; q += SL)
      surface_face<T, OP>(A, g, A.ent[q], pe, acc);
  }
#pragma unroll
  for (int o = SL / 2; o > 0; o >>= 1)
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] += __shfl_xor(acc[i], o);
  if (k < A.nsn && sub == 0) {
    if (OP == OP_ENERGY) {
#pragma unroll
      for (int i = 0; i < 3; ++i) e += 0.5 * double(A.u[3 * int64_t(g) + i]) * double(acc[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) A.fs[3 * int64_t(g) + i] = acc[i];
    }
  }
  if (OP == OP_ENERGY) {
    double v = e;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = 0.0;
      for (int w = 0; w < NT / 64; ++w) r += sh[w];
      A.red[blockIdx.x] = r;
    }
  }
}

// Quadratic faces (6 nodes: vertices, then the midpoints of edges (0,1),
// (1,2), (0,2)) of a second-order mesh: follower pressure and springs (with
// dashpots).  Node a of a face gains, for the pressure,
//   pe int N_a (x_xi x x_eta) dxi deta     (residual),
//   pl int N_a (v_xi x x_eta + x_xi x v_eta) (Jacobian action),
// over the reference triangle by the 6-point degree-4 rule of Dunavant
// (exact: the integrand has degree 4), and for the springs
// sum_b M_ab K w_b with the exact face mass M = 2A/360 [6 -1 -1 0 -4 0; ...]
// (vertex-vertex 6 / -1, vertex-midpoint 0 on its edges and -4 opposite,
// midpoint-midpoint 32 / 16).  The pressure adds nothing to the diagonal:
// (e_i x y)_i = 0.
__constant__ double D6_L[6][3] = {
    {0.445948490915965, 0.445948490915965, 0.108103018168070},
    {0.445948490915965, 0.108103018168070, 0.445948490915965},
    {0.108103018168070, 0.445948490915965, 0.445948490915965},
    {0.091576213509771, 0.091576213509771, 0.816847572980459},
    {0.091576213509771, 0.816847572980459, 0.091576213509771},
    {0.816847572980459, 0.091576213509771, 0.091576213509771}};
__constant__ double D6_W[6] = {0.223381589678011, 0.223381589678011, 0.223381589678011,
                               0.109951743655322, 0.109951743655322, 0.109951743655322};
__constant__ double M6_REF[6][6] = {{6, -1, -1, 0, -4, 0},   {-1, 6, -1, 0, 0, -4},
                                    {-1, -1, 6, -4, 0, 0},   {0, 0, -4, 32, 16, 16},
                                    {-4, 0, 0, 16, 32, 16},  {0, -4, 0, 16, 16, 32}};

// value and (xi, eta) derivatives of the face's shape function a at
// barycentric (L0, L1, L2), xi = L1, eta = L2
__device__ __forceinline__ void tri6_shape(int a, const double L[3], double &N, double &dx,
                                           double &de) {
  const double dL[3][2] = {{-1.0, -1.0}, {1.0, 0.0}, {0.0, 1.0}};
  if (a < 3) {
    N = L[a] * (2.0 * L[a] - 1.0);
    dx = (4.0 * L[a] - 1.0) * dL[a][0];
    de = (4.0 * L[a] - 1.0) * dL[a][1];
  } else {
    const int p = a == 3 ? 0 : (a == 4 ? 1 : 0), q = a == 3 ? 1 : 2;
    N = 4.0 * L[p] * L[q];
    dx = 4.0 * (L[p] * dL[q][0] + L[q] * dL[p][0]);
    de = 4.0 * (L[p] * dL[q][1] + L[q] * dL[p][1]);
  }
}

template <typename T, int OP>
__global__ __launch_bounds__(NT) void k_surface6(SurfArgs<T> A) {
  __shared__ double sh[NT / 64];
  if (A.skip && A.skip[0] != 0) return;
  const int64_t k = int64_t(blockIdx.x) * NT + threadIdx.x;
  double e = 0.0;
  if (k < A.nsn) {
    const int32_t g = A.node[k];
    T acc[3] = {T(0), T(0), T(0)};
    const T pe = OP == OP_JV ? T(A.plin[0]) : T(A.p);
    for (int q = A.ptr[k]; q < A.ptr[k + 1]; ++q) {
      const int32_t f = A.ent[q];
      int32_t n[6];
#pragma unroll
      for (int a = 0; a < 6; ++a) n[a] = A.tri[6 * int64_t(f) + a];
      int me = 0;
#pragma unroll
      for (int a = 0; a < 6; ++a)
        if (n[a] == g) me = a;
      const uint32_t fm = (OP == OP_JV && !A.nomask) ? A.fmask[f] : 0u;
      if (f < A.npf) {
        if (OP != OP_RES && OP != OP_JV) continue;
        const T *Xf = A.pgeo + 18 * int64_t(f);
        T x[6][3], w[6][3];
#pragma unroll
        for (int a = 0; a < 6; ++a)
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            x[a][i] = Xf[3 * a + i] + A.u[3 * int64_t(n[a]) + i];
            if (OP == OP_JV) w[a][i] = ((fm >> (3 * a + i)) & 1u) ? T(0) : A.v[3 * int64_t(n[a]) + i];
          }
        for (int qp = 0; qp < 6; ++qp) {
          const double L[3] = {D6_L[qp][0], D6_L[qp][1], D6_L[qp][2]};
          T xx[3] = {T(0), T(0), T(0)}, xe[3] = {T(0), T(0), T(0)};
          T vx[3] = {T(0), T(0), T(0)}, ve[3] = {T(0), T(0), T(0)};
          double Nme = 0.0;
#pragma unroll
          for (int a = 0; a < 6; ++a) {
            double N, dx, de;
            tri6_shape(a, L, N, dx, de);
            if (a == me) Nme = N;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              xx[i] += T(dx) * x[a][i];
              xe[i] += T(de) * x[a][i];
              if (OP == OP_JV) {
                vx[i] += T(dx) * w[a][i];
                ve[i] += T(de) * w[a][i];
              }
            }
          }
          // reference area 1/2 times the rule's weight
          const T s = pe * T(0.5 * D6_W[qp] * Nme);
          if (OP == OP_RES) {
            cross_acc(xx, xe, s, acc);
          } else {
            cross_acc(vx, xe, s, acc);
            cross_acc(xx, ve, s, acc);
          }
        }
      } else {
        const T *R = A.rgeo + 4 * int64_t(f - A.npf - A.ntf);
        const T N[3] = {R[0], R[1], R[2]};
        const T area = R[3];
        const T kpar = T(A.kpar), dk = T(A.kperp - A.kpar);
        const T kpe = A.damp ? T(A.kpar + A.cv * A.cpar) : kpar;
        const T dke = A.damp ? T(A.kperp - A.kpar + A.cv * (A.cperp - A.cpar)) : dk;
        const T m2 = T(2) * area / T(360);
        if (OP == OP_DIAG) {
#pragma unroll
          for (int i = 0; i < 3; ++i) acc[i] += m2 * T(M6_REF[me][me]) * (kpe + dke * N[i] * N[i]);
        } else if (OP == OP_RES || OP == OP_JV || OP == OP_ENERGY) {
          const T *wv = OP == OP_JV ? A.v : A.u;
          const T kw = OP == OP_JV ? kpe : kpar, dw = OP == OP_JV ? dke : dk;
#pragma unroll
          for (int b = 0; b < 6; ++b) {
            const T m = m2 * T(M6_REF[me][b]);
            const int64_t nb = int64_t(n[b]);
            T wb[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) wb[i] = ((fm >> (3 * b + i)) & 1u) ? T(0) : wv[3 * nb + i];
            const T nw = N[0] * wb[0] + N[1] * wb[1] + N[2] * wb[2];
#pragma unroll
            for (int i = 0; i < 3; ++i) acc[i] += m * (kw * wb[i] + dw * nw * N[i]);
            if (OP == OP_RES && A.damp) {
              T z[3];
#pragma unroll
              for (int i = 0; i < 3; ++i)
                z[i] = T(A.vt[3 * nb + i] + A.cv * (double(A.u[3 * nb + i]) - A.ut[3 * nb + i]));
              const T nz = N[0] * z[0] + N[1] * z[1] + N[2] * z[2];
              const T cpar = T(A.cpar), dc = T(A.cperp - A.cpar);
#pragma unroll
              for (int i = 0; i < 3; ++i) acc[i] += m * (cpar * z[i] + dc * nz * N[i]);
            }
          }
        }
      }
    }
    if (OP == OP_ENERGY) {
#pragma unroll
      for (int i = 0; i < 3; ++i) e += 0.5 * double(A.u[3 * int64_t(g) + i]) * double(acc[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) A.fs[3 * int64_t(g) + i] = acc[i];
    }
  }
  if (OP == OP_ENERGY) {
    double v = e;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = 0.0;
      for (int w = 0; w < NT / 64; ++w) r += sh[w];
      A.red[blockIdx.x] = r;
    }
  }
}

__global__ void k_set_scalar(double *dst, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = v;
}

template <typename T>
void launch_surface(Ctx *c, int op, const T *u, const T *v, T *fs, double *red, const T *pgeo,
                    const T *rgeo) {
  const Ctx::Surf &S = c->surf;
  SurfArgs<T> A;
  A.nsn = S.nsn;
  A.npf = S.npf;
  A.ntf = S.ntf;
  A.node = S.node;
  A.ptr = S.ptr;
  A.ent = S.ent;
  A.tri = S.tri;
  A.fmask = S.fmask;
  A.pgeo = pgeo;
  A.rgeo = rgeo;
  A.p = c->load_scale * S.p;
  A.s = c->load_scale;
  A.plin = S.plin;
  for (int i = 0; i < 3; ++i) A.tf[i] = S.tf[i];
  A.kperp = S.kperp;
  A.kpar = S.kpar;
  A.damp = damping_on(c) ? 1 : 0;
  A.cperp = S.cperp;
  A.cpar = S.cpar;
  A.cv = c->inr.cv;
  A.vt = c->inr.vt;
  A.ut = c->inr.ut;
  A.u = u;
  A.v = v;
  A.fs = fs;
  A.red = red;
  A.skip = c->elem_skip;
  A.nomask = (op == OP_JV && c->jv_nomask) ? 1 : 0;
  const int grid = int((S.nsn + NT - 1) / NT);
  if (S.fv == 6) {
    switch (op) {
      case OP_RES:
        hipLaunchKernelGGL((k_surface6<T, OP_RES>), dim3(grid), dim3(NT), 0, c->stream, A);
        break;
      case OP_JV:
        hipLaunchKernelGGL((k_surface6<T, OP_JV>), dim3(grid), dim3(NT), 0, c->stream, A);
        break;
      case OP_DIAG:
        hipLaunchKernelGGL((k_surface6<T, OP_DIAG>), dim3(grid), dim3(NT), 0, c->stream, A);
        break;
      default:
        hipLaunchKernelGGL((k_surface6<T, OP_ENERGY>), dim3(grid), dim3(NT), 0, c->stream, A);
        break;
    }
    return;
  }
  constexpr int SL = 8;
  const int grid8 = int((SL * S.nsn + NT - 1) / NT);
  switch (op) {
    case OP_RES:
      hipLaunchKernelGGL((k_surface<T, OP_RES, SL>), dim3(grid8), dim3(NT), 0, c->stream, A);
      break;
    case OP_JV:
      hipLaunchKernelGGL((k_surface<T, OP_JV, SL>), dim3(grid8), dim3(NT), 0, c->stream, A);
      break;
    case OP_DIAG:
      hipLaunchKernelGGL((k_surface<T, OP_DIAG, SL>), dim3(grid8), dim3(NT), 0, c->stream, A);
      break;
    case OP_ODIAG:
      hipLaunchKernelGGL((k_surface<T, OP_ODIAG, SL>), dim3(grid8), dim3(NT), 0, c->stream, A);
      break;
    default:
      hipLaunchKernelGGL((k_surface<T, OP_ENERGY, 1>), dim3(grid), dim3(NT), 0, c->stream, A);
      break;
  }
}

template <typename T>
T *bupload(Ctx *c, const std::vector<T> &h, hipError_t *e) {
  T *d = static_cast<T *>(dalloc(c, std::max<size_t>(h.size(), 1) * sizeof(T)));
  if (!d) {
    *e = hipErrorOutOfMemory;
    return nullptr;
  }
  c->surf.allocs.push_back(d);
  if (!h.empty()) {
    const hipError_t r =
        hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream);
    if (r != hipSuccess) *e = r;
  }
  return d;
}

}  // namespace

void free_surface(Ctx *c) {
  Ctx::Surf &S = c->surf;
  for (void *p : S.allocs) dfree(c, p);
  S.allocs.clear();
  S.nsn = 0;
  S.npf = S.ntf = S.nrf = 0;
  S.node = S.ptr = S.ent = S.tri = nullptr;
  S.fmask = nullptr;
  S.pgeo64 = S.rgeo64 = S.plin = S.fs64 = nullptr;
  S.pgeo32 = S.rgeo32 = S.fs32 = nullptr;
}

nle_status build_surface(Ctx *c) {
  Ctx::Surf &S = c->surf;
  drop_graph(c);
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  free_surface(c);
  const int64_t npf0 = int64_t(S.h_ptri.size() / 3), ntf = int64_t(S.h_ttri.size() / 3);
  const int64_t nrf = int64_t(S.h_rtri.size() / 3);
  const int64_t npf = npf0 + ntf;  // faces carrying reference coordinates
  if (npf + nrf == 0) return NLE_OK;
  if (npf + nrf >= (int64_t(1) << 31) / 3) return fail(c, NLE_E_UNSUPPORTED, "too many faces");
  const int64_t nn = c->m.n_nodes;
  const double *X = c->m.h_X.data();
  std::vector<int32_t> tri3(S.h_ptri);
  tri3.insert(tri3.end(), S.h_ttri.begin(), S.h_ttri.end());
  tri3.insert(tri3.end(), S.h_rtri.begin(), S.h_rtri.end());
  // quadratic meshes: each face gains the midpoints of its edges (0,1), (1,2), (0,2)
  const int fv = c->mixed ? 6 : 3;
  std::vector<int32_t> tri;
  if (fv == 3) {
    tri = tri3;
  } else {
    if (ntf > 0) return fail(c, NLE_E_UNSUPPORTED, "follower traction needs a P1 mesh");
    std::unordered_map<uint64_t, int32_t> mid;
    const std::vector<int32_t> &cn = c->mx.h_conn;
    static const int ea[6] = {0, 1, 0, 0, 1, 2}, eb[6] = {1, 2, 2, 3, 3, 3};
    for (size_t e0 = 0; e0 + 9 < cn.size(); e0 += 10)
      for (int q = 0; q < 6; ++q) {
        const uint32_t va = uint32_t(cn[e0 + ea[q]]), vb = uint32_t(cn[e0 + eb[q]]);
        mid[(uint64_t(std::min(va, vb)) << 32) | std::max(va, vb)] = cn[e0 + 4 + q];
      }
    const int pa[3] = {0, 1, 0}, pb[3] = {1, 2, 2};
    for (size_t f = 0; f < tri3.size() / 3; ++f) {
      for (int a = 0; a < 3; ++a) tri.push_back(tri3[3 * f + a]);
      for (int q = 0; q < 3; ++q) {
        const uint32_t va = uint32_t(tri3[3 * f + pa[q]]), vb = uint32_t(tri3[3 * f + pb[q]]);
        auto it = mid.find((uint64_t(std::min(va, vb)) << 32) | std::max(va, vb));
        if (it == mid.end()) return fail(c, NLE_E_INVAL, "face edge is not an element edge");
        tri.push_back(it->second);
      }
    }
  }
  // incident faces of each node (CSR over nodes, faces in increasing order)
  std::vector<int32_t> cnt(nn + 1, 0);
  for (int32_t v : tri) cnt[v + 1] += 1;
  std::vector<int32_t> fnode, fptr(1, 0), fent;
  std::vector<int64_t> start(nn + 1, 0);
  for (int64_t g = 0; g < nn; ++g) start[g + 1] = start[g] + cnt[g + 1];
  std::vector<int32_t> all(start[nn]);
  std::vector<int64_t> pos(start.begin(), start.end() - 1);
  const int64_t nf = npf + nrf;
  for (int64_t f = 0; f < nf; ++f)
    for (int a = 0; a < fv; ++a) {
      const int32_t v = tri[fv * f + a];
      // a face listing a node twice would add it twice: rejected
      for (int b = 0; b < a; ++b)
        if (tri[fv * f + b] == v) return fail(c, NLE_E_BADMESH, "degenerate surface triangle");
      all[pos[v]++] = int32_t(f);
    }
  for (int64_t g = 0; g < nn; ++g) {
    if (start[g + 1] == start[g]) continue;
    fnode.push_back(int32_t(g));
    for (int64_t q = start[g]; q < start[g + 1]; ++q) fent.push_back(all[q]);
    fptr.push_back(int32_t(fent.size()));
  }
  std::vector<double> pg(3 * fv * npf), rg(4 * nrf);
  for (int64_t f = 0; f < npf; ++f)
    for (int a = 0; a < fv; ++a)
      for (int i = 0; i < 3; ++i) pg[3 * fv * f + 3 * a + i] = X[3 * int64_t(tri[fv * f + a]) + i];
  for (int64_t r = 0; r < nrf; ++r) {
    const int32_t *t = &tri[fv * (npf + r)];
    double e1[3], e2[3];
    for (int i = 0; i < 3; ++i) {
      e1[i] = X[3 * int64_t(t[1]) + i] - X[3 * int64_t(t[0]) + i];
      e2[i] = X[3 * int64_t(t[2]) + i] - X[3 * int64_t(t[0]) + i];
    }
    const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                         e1[0] * e2[1] - e1[1] * e2[0]};
    const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(l > 0.0)) return fail(c, NLE_E_BADMESH, "zero-area spring triangle");
    for (int i = 0; i < 3; ++i) rg[4 * r + i] = n[i] / l;
    rg[4 * r + 3] = 0.5 * l;
  }
  std::vector<float> pg32(pg.begin(), pg.end()), rg32(rg.begin(), rg.end());
  hipError_t e = hipSuccess;
  S.fv = fv;
  S.npf = int32_t(npf0);
  S.ntf = int32_t(ntf);
  S.nrf = int32_t(nrf);
  S.nsn = int64_t(fnode.size());
  S.node = bupload(c, fnode, &e);
  S.ptr = bupload(c, fptr, &e);
  S.ent = bupload(c, fent, &e);
  S.tri = bupload(c, tri, &e);
  const std::vector<uint32_t> fm0(nf, 0u);
  S.fmask = bupload(c, fm0, &e);
  S.pgeo64 = bupload(c, pg, &e);
  S.pgeo32 = bupload(c, pg32, &e);
  S.rgeo64 = bupload(c, rg, &e);
  S.rgeo32 = bupload(c, rg32, &e);
  S.plin = static_cast<double *>(dalloc(c, 256));
  S.fs64 = static_cast<double *>(dalloc(c, size_t(3 * nn) * 8));
  S.fs32 = static_cast<float *>(dalloc(c, size_t(3 * nn) * 4));
  for (void *p : {(void *)S.plin, (void *)S.fs64, (void *)S.fs32}) {
    if (!p) e = hipErrorOutOfMemory;
    S.allocs.push_back(p);
  }
  if (e == hipErrorOutOfMemory) {
    free_surface(c);
    return fail(c, NLE_E_OOM, "device allocation failed");
  }
  if (e != hipSuccess) {
    free_surface(c);
    return fail(c, NLE_E_HIP, std::string("surface upload: ") + hipGetErrorString(e));
  }
  // entries off the face nodes stay zero for good
  NLE_HIP(c, hipMemsetAsync(S.fs64, 0, size_t(3 * nn) * 8, c->stream));
  NLE_HIP(c, hipMemsetAsync(S.fs32, 0, size_t(3 * nn) * 4, c->stream));
  NLE_HIP(c, hipMemsetAsync(S.plin, 0, 16, c->stream));
  S.h_tri = tri;
  c->lin64 = c->lin32 = c->lc_valid = false;
  return upload_surface_masks(c);
}

nle_status upload_surface_masks(Ctx *c) {
  Ctx::Surf &S = c->surf;
  if (S.nsn == 0) return NLE_OK;
  const int fv = S.fv;
  const int64_t nf = int64_t(S.h_tri.size() / fv);
  std::vector<uint32_t> fm(nf, 0u);
  for (int64_t f = 0; f < nf; ++f)
    for (int a = 0; a < fv; ++a)
      fm[f] |= uint32_t(c->h_mask[S.h_tri[fv * f + a]] & 7u) << (3 * a);
  NLE_HIP(c, hipMemcpyAsync(S.fmask, fm.data(), fm.size() * 4, hipMemcpyHostToDevice, c->stream));
  NLE_HIP(c, hipStreamSynchronize(c->stream));
  return NLE_OK;
}

hipError_t surf_set_linear_pressure(Ctx *c) {
  if (c->surf.nsn == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, c->stream, c->surf.plin,
                     c->load_scale * c->surf.p);
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, c->stream, c->surf.plin + 1,
                     c->load_scale);
  return hipGetLastError();
}

void *surf_apply(Ctx *c, int op, int prec, const void *u, const void *v, int *n_red,
                 hipError_t *err, double *red) {
  const Ctx::Surf &S = c->surf;
  *err = hipSuccess;
  if (S.nsn == 0) {
    if (n_red) *n_red = 0;
    return nullptr;
  }
  const int grid = int((S.nsn + NT - 1) / NT);
  if (n_red) *n_red = op == OP_ENERGY ? grid : 0;
  void *fs;
  if (prec == NLE_FP32) {
    fs = S.fs32;
    launch_surface<float>(c, op, static_cast<const float *>(u), static_cast<const float *>(v),
                          S.fs32, red, S.pgeo32, S.rgeo32);
  } else {
    fs = S.fs64;
    launch_surface<double>(c, op, static_cast<const double *>(u), static_cast<const double *>(v),
                           S.fs64, red, S.pgeo64, S.rgeo64);
  }
  *err = hipGetLastError();
  return fs;
}

}  // namespace nle
