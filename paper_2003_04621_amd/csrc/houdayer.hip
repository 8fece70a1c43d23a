// houdayer.hip -- Houdayer cluster move in overlap space (Sec. 2.4, Eq. (10)),
// one workgroup per (sample, temperature) pair.
//
// The pair's two replicas a, b are read into LDS as row words; the overlap
// word Q = W_a ^ W_b has a bit set where q_i = s_i^a s_i^b = -1.  The seed is
// the m-th set bit in increasing site order (per-thread row chunks, a prefix
// sum over chunks, then a walk along x0 inside the row).  The cluster grows
// by bit-parallel flood fill: C_c |= Q_c & (union of the neighbour words of
// C_{1-c}), alternating colours until no word changes -- label propagation
// of the seed's single label, one row word (H sites) per operation.  The
// energy change of replica a is delta = 2 (#boundary bonds - 2 #unsatisfied
// boundary bonds), counted on colour-0 words where every bond has one end.
#include "device.h"
#include "kernels.h"

namespace ptsg {

template <int D>
__global__ void __launch_bounds__(256) k_houdayer(Geo g, void* spins, const uint32_t* __restrict__ jw,
                                                  int32_t* __restrict__ E,
                                                  const int32_t* __restrict__ sot, DevCounters* ctr) {
  extern __shared__ uint32_t lds[];
  const int T = blockDim.x, t = threadIdx.x;
  uint32_t* A = lds;                      // replica a, both colours
  uint32_t* Q = A + 2 * g.NR;             // overlap words (later replica b)
  uint32_t* Cl = Q + 2 * g.NR;            // cluster words
  uint32_t* pre = Cl + 2 * g.NR;          // [T] chunk counts -> prefix sums
  __shared__ uint32_t n_minus;
  __shared__ int delta_acc;

  const uint32_t v = load_counter(&ctr->v);
  const int pair = blockIdx.x;  // s*NT + k
  const int s = pair / g.NT, k = pair - s * g.NT;
  const int a = sot[((size_t)s * 2 + 0) * g.NT + k];
  const int b = g.NT + sot[((size_t)s * 2 + 1) * g.NT + k];
  const size_t lat_a = (size_t)s * g.nslot + a, lat_b = (size_t)s * g.nslot + b;

  load_lattice(g, spins, lat_a, A, t, T);
  load_lattice(g, spins, lat_b, Q, t, T);
  if (t == 0) delta_acc = 0;
  __syncthreads();
  for (int w = t; w < 2 * g.NR; w += T) {
    Q[w] ^= A[w];
    Cl[w] = 0;
  }
  __syncthreads();

  // q = -1 counts per contiguous row chunk
  const int chunk = (g.NR + T - 1) / T;
  const int r_begin = t * chunk, r_end = min(g.NR, r_begin + chunk);
  uint32_t cnt = 0;
  for (int R = r_begin; R < r_end; ++R) cnt += __popc(Q[R]) + __popc(Q[g.NR + R]);
  pre[t] = cnt;
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    for (int i = 0; i < T; ++i) {
      const uint32_t c = pre[i];
      pre[i] = run;
      run += c;
    }
    n_minus = run;
  }
  __syncthreads();
  const uint32_t n = n_minus;
  if (n > 0) {
    const Ctr4 r = philox10(Ctr4{(uint32_t)k, v, 0u, (kTagHou << 28) | (uint32_t)s}, g.key0, g.key1);
    const uint64_t r64 = (uint64_t)r.x | ((uint64_t)r.y << 32);
    const uint32_t m = (uint32_t)__umul64hi(r64, (uint64_t)n);
    if (m >= pre[t] && m < pre[t] + cnt) {
      uint32_t rem = m - pre[t];
      for (int R = r_begin; R < r_end; ++R) {
        const uint32_t cr = __popc(Q[R]) + __popc(Q[g.NR + R]);
        if (rem >= cr) {
          rem -= cr;
          continue;
        }
        const RowNb q = row_nb(g, R);
        for (int x0 = 0; x0 < g.L; ++x0) {
          const int c = (x0 & 1) ^ q.p0;
          const uint32_t bit = (Q[c * g.NR + R] >> (x0 >> 1)) & 1u;
          if (bit) {
            if (rem == 0) {
              Cl[c * g.NR + R] = 1u << (x0 >> 1);
              break;
            }
            --rem;
          }
        }
        break;
      }
    }
    __syncthreads();

    // flood fill
    int any;
    do {
      int changed = 0;
      for (int c = 0; c < 2; ++c) {
        const uint32_t* X = Cl + (1 - c) * g.NR;
        for (int R = t; R < g.NR; R += T) {
          const uint32_t qw = Q[c * g.NR + R];
          if (!qw) continue;
          const RowNb q = row_nb(g, R);
          const int p = (c + q.x1 + q.x2) & 1;
          uint32_t n0, n1;
          x0_neighbours(g, X[R], p, n0, n1);
          uint32_t nb = n0 | n1 | X[q.r1p] | X[q.r1m];
          if (D == 3) nb |= X[q.r2p] | X[q.r2m];
          const uint32_t old = Cl[c * g.NR + R];
          const uint32_t nw = old | (qw & nb);
          if (nw != old) {
            Cl[c * g.NR + R] = nw;
            changed = 1;
          }
        }
        if (c == 0) __syncthreads();
      }
      any = __syncthreads_or(changed);
    } while (any);

    // energy change of replica a on the colour-0 words
    const uint32_t* jw0 = jw + (size_t)s * 2 * 2 * D * g.NR;
    int cross = 0, cross_u = 0;
    for (int R = t; R < g.NR; R += T) {
      const RowNb q = row_nb(g, R);
      const int p = q.p0;
      const uint32_t C0 = Cl[R], A0 = A[R];
      const uint32_t* C1 = Cl + g.NR;
      const uint32_t* A1 = A + g.NR;
      uint32_t c0p, c0m, a0p, a0m;
      x0_neighbours(g, C1[R], p, c0p, c0m);
      x0_neighbours(g, A1[R], p, a0p, a0m);
      uint32_t X[2 * D], U[2 * D];
      X[0] = C0 ^ c0p;
      U[0] = A0 ^ a0p ^ jw0[0 * (size_t)g.NR + R];
      X[1] = C0 ^ c0m;
      U[1] = A0 ^ a0m ^ jw0[1 * (size_t)g.NR + R];
      X[2] = C0 ^ C1[q.r1p];
      U[2] = A0 ^ A1[q.r1p] ^ jw0[2 * (size_t)g.NR + R];
      X[3] = C0 ^ C1[q.r1m];
      U[3] = A0 ^ A1[q.r1m] ^ jw0[3 * (size_t)g.NR + R];
      if (D == 3) {
        X[4] = C0 ^ C1[q.r2p];
        U[4] = A0 ^ A1[q.r2p] ^ jw0[4 * (size_t)g.NR + R];
        X[5] = C0 ^ C1[q.r2m];
        U[5] = A0 ^ A1[q.r2m] ^ jw0[5 * (size_t)g.NR + R];
      }
#pragma unroll
      for (int dd = 0; dd < 2 * D; ++dd) {
        cross += __popc(X[dd]);
        cross_u += __popc(X[dd] & U[dd]);
      }
    }
    atomicAdd(&delta_acc, 2 * (cross - 2 * cross_u));
    __syncthreads();

    // exchange the replicas on the cluster: a' = a ^ C, b' = Q ^ a'
    for (int w = t; w < 2 * g.NR; w += T) {
      const uint32_t an = A[w] ^ Cl[w];
      A[w] = an;
      Q[w] ^= an;
    }
    __syncthreads();
    store_lattice(g, spins, lat_a, A, t, T, Cl);
    store_lattice(g, spins, lat_b, Q, t, T, Cl);
    if (t == 0) {
      E[lat_a] += delta_acc;
      E[lat_b] -= delta_acc;
    }
  }
}

hipError_t launch_houdayer(const Geo& g, void* spins, const uint32_t* jw, int32_t* E,
                           const int32_t* sot, DevCounters* ctr, hipStream_t st) {
  int threads = ((g.NR + 63) / 64) * 64;
  if (threads > 256) threads = 256;
  const size_t lds = sizeof(uint32_t) * (6 * (size_t)g.NR + threads);
  const unsigned blocks = (unsigned)(g.S * g.NT);
  if (g.d == 3) {
    if (lds > 65536)
      { const hipError_t ea = hipFuncSetAttribute((const void*)k_houdayer<3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); if (ea != hipSuccess) return ea; }
    hipLaunchKernelGGL(k_houdayer<3>, dim3(blocks), dim3(threads), lds, st, g, spins, jw, E, sot, ctr);
  } else {
    if (lds > 65536)
      { const hipError_t ea = hipFuncSetAttribute((const void*)k_houdayer<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); if (ea != hipSuccess) return ea; }
    hipLaunchKernelGGL(k_houdayer<2>, dim3(blocks), dim3(threads), lds, st, g, spins, jw, E, sot, ctr);
  }
  return hipGetLastError();
}

}  // namespace ptsg
