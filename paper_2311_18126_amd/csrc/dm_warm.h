// dm_warm.h -- step-start guess of the Newton solve inside the step kernel (device code of
// dm_kernels.hip).  Every system predicts its own nodes' displacement over the step at the
// start of each step, so warm-started stepping keeps the one persistent launch per call.
//
// Guesses (the positions handed to Newton; Newton still judges convergence, and a failed
// guess restarts from x_n):
//   mode 1: x_n + dt v_n (explicit predictor);
//   mode 3: x_n + dt (v_n + a_n), a_n = v_n - v_{n-1} (second-order extrapolation);
//   mode 4: x_n + dt (v_n + a_n + j_n), j_n = a_n - a_{n-1} (third-order extrapolation);
//   mode 2: mode 4 plus the network's correction s * y, y = MLP(standardised features), scaled
//           by the share of the time step that the Newton unknown covers (a substep of adaptive
//           halving; half the step for the midpoint state of the implicit-midpoint rule).
// The network runs on the matrix cores in bfloat16 with float32 accumulation, rounded at the
// same points and accumulated in the same order as the batch kernels of dm_mlp.hip.
#pragma once
#include "dm_bf16.h"

// Chain node (c, k) of row i of system S (rows run over the system's chains in order).
__device__ __forceinline__ void system_row(const DmDev DM_C& D, const DmSystem DM_C& S, int i, int& c, int& k) {
  c = S.chain0;
  k = i;
  while (k >= D.chain[c].n_nodes) { k -= D.chain[c].n_nodes; ++c; }
}

// The 26 raw features of node k of chain ch (missing neighbours of a rod end replicated):
// v_{k-1} - v_k, v_{k+1} - v_k, v_k, a_k = v_k - v_prev_k, x_{k-1} - 2 x_k + x_{k+1} (step-start
// positions), log10 E, radius, mean rest length of the node's edges, natural curvature at the
// node in 1/m (nearest interior node at the ends), j_k = a_k - (v_prev_k - v_prev2_k) (the
// change of the velocity change), a_{k-1} - 2 a_k + a_{k+1}.
__device__ __forceinline__ void row_features(const DmDev DM_C& D, const DmChain& ch, int k, double (&f)[DM_NET_IN]) {
  const int NN = D.n_nodes_tot, NS = D.n_st_tot, N = ch.n_nodes;
  const int n0 = D.chain_node[ch.node_tab + k];
  const int nm = D.chain_node[ch.node_tab + (k >= 1 ? k - 1 : k)];
  const int np = D.chain_node[ch.node_tab + (k <= N - 2 ? k + 1 : k)];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double vi = D.v[q * NN + n0], ai = vi - D.vprev[q * NN + n0];
    f[q] = D.v[q * NN + nm] - vi;
    f[3 + q] = D.v[q * NN + np] - vi;
    f[6 + q] = vi;
    f[9 + q] = ai;
    f[12 + q] = D.x0[q * NN + nm] - 2.0 * D.x0[q * NN + n0] + D.x0[q * NN + np];
    f[20 + q] = ai - (D.vprev[q * NN + n0] - D.vprev2[q * NN + n0]);
    f[23 + q] = (D.v[q * NN + nm] - D.vprev[q * NN + nm]) - 2.0 * ai + (D.v[q * NN + np] - D.vprev[q * NN + np]);
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) f[15 + q] = D.nconst[(size_t)(ch.node_tab + k) * 3 + q];
  f[18] = f[19] = 0.0;
  if (N >= 3) {
    const int kc = k < 1 ? 1 : (k > N - 2 ? N - 2 : k);
    const int s = ch.st_off + kc - 1;
    f[18] = D.kbar[s] / D.Vbar[s];
    f[19] = D.kbar[NS + s] / D.Vbar[s];
  }
}

// Displacement component q of node k of chain ch without the network: dt v_n (mode 1),
// dt (v_n + a_n) (mode 3), dt (v_n + a_n + j_n) (modes 2 and 4), dt the Newton step of the
// (sub)step.
__device__ __forceinline__ double base_guess(const DmStepArgs DM_C& A, double dt, const DmChain& ch, int k, int q) {
  const DmDev DM_C& D = A.d;
  const int NN = D.n_nodes_tot;
  const int n0 = D.chain_node[ch.node_tab + k];
  const double v = D.v[q * NN + n0];
  double d = dt * v;
  if (A.warm >= 2) {
    const double vp = D.vprev[q * NN + n0], a = v - vp;
    d += dt * a;
    if (A.warm != 3) d += dt * (a - (vp - D.vprev2[q * NN + n0]));
  }
  return d;
}

// Hand displacement d of DOF q of node k of chain ch to Newton (positions of free nodes, by
// the chain that owns the node), or store it to out[row][q] (prediction only).
__device__ __forceinline__ void put_guess(const DmStepArgs DM_C& A, const DmChain& ch, int k, int q, double d,
                                          double DM_G* out) {
  const DmDev DM_C& D = A.d;
  if (out) { out[(size_t)(ch.node_tab + k) * 3 + q] = d; return; }
  const int NN = D.n_nodes_tot;
  const int n0 = D.chain_node[ch.node_tab + k];
  if (D.node_owner[n0] != ch.global_id || D.cfix[ch.dof_off + 4 * k + q]) return;
  D.x[q * NN + n0] = D.x0[q * NN + n0] + d;
}

__device__ __forceinline__ dm_bf16x8 ld_bf16x8(const unsigned short DM_C* p) {
  return *(const dm_bf16x8 DM_C*)p;
}

// Input fragment of one lane: standardised features 8g .. 8g+7 of system row i (zero beyond
// the system's rows and past the last feature), rounded to bfloat16.
__device__ __forceinline__ dm_bf16x8 input_fragment(const DmStepArgs DM_C& A, const DmSystem DM_C& S, int i, int g) {
  const DmDev DM_C& D = A.d;
  const DmNetView DM_C& W = A.net;
  const bool valid = i < S.chain_nodes;
  int c, k;
  system_row(D, S, valid ? i : 0, c, k);
  const DmChain ch = D.chain[c];
  double f[DM_NET_IN];
  row_features(D, ch, k, f);
  dm_bf16x8 a;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int q = 8 * g + j;
    const bool real = valid & (q < DM_NET_IN);
    const int qc = real ? q : 0;
    // constant indices only (j is unrolled), so f stays in registers
    const double fv = g == 0 ? f[j] : (g == 1 ? f[8 + j] : (g == 2 ? f[16 + j] : (24 + j < DM_NET_IN ? f[(24 + j) % DM_NET_IN] : 0.0)));
    const unsigned short h = real ? dm_bf16_bits((float)((fv - W.mean[qc]) / W.sd[qc])) : (unsigned short)0;
    a[j] = __builtin_bit_cast(__bf16, h);
  }
  return a;
}

// ReLU(acc + bias) rounded to bfloat16 into activation rows 16 rt + 4 (l / 16) + j, columns
// 64 cb + 16 ct + l % 16 of buffer h.
__device__ __forceinline__ void store_block(const dm_f32x4 (&acc)[DM_NET_RT][4], const float DM_C* bias, int cb,
                                            unsigned short DM_L* h, int lane) {
  const int lr = lane & 15, g = lane >> 4;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int n = 64 * cb + 16 * ct + lr;
    const float b = bias[n];
#pragma unroll
    for (int rt = 0; rt < DM_NET_RT; ++rt)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        h[(16 * rt + 4 * g + j) * DM_NET_LDS_ROW + n] = dm_bf16_bits(fmaxf(acc[rt][ct][j] + b, 0.0f));
  }
}

__device__ __forceinline__ dm_bf16x8 lds_fragment(const unsigned short DM_L* h, int row, int col) {
  return *(const dm_bf16x8 DM_L*)(h + row * DM_NET_LDS_ROW + col);
}

// Products of one 32-wide reduction step k0 of layer 2 for every row tile and the four
// column tiles whose weight fragments are b.
__device__ __forceinline__ void layer2_step(dm_f32x4 (&acc)[DM_NET_RT][4], const dm_bf16x8 (&b)[4],
                                            const unsigned short DM_L* P, int k0, int lane) {
  const int lr = lane & 15, g = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < DM_NET_RT; ++rt) {
    const dm_bf16x8 a = lds_fragment(P, 16 * rt + lr, k0 + 8 * g);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = dm_mfma_bf16(a, b[ct], acc[rt][ct]);
  }
}

// The network's guess for system rows row0 .. row0 + 16 DM_NET_RT - 1, by the whole workgroup (uniform
// control flow: every thread reaches the barriers).  Row tiles of 16 and column blocks of 64
// are dealt to the first DM_NET_WAVES wavefronts; each output accumulates over the reduction
// index in ascending order, one matrix-core chain per tile, as in the batch kernels.
// LDS: P holds layer 1's activations, Q the inputs and then layer 2's activations.
__device__ __forceinline__ void network_block(const DmStepArgs DM_C& A, double dt, const DmSystem DM_C& S, int row0,
                                              unsigned short DM_L* P, unsigned short DM_L* Q, double DM_G* out) {
  const DmDev DM_C& D = A.d;
  const DmNetView DM_C& W = A.net;
  const int lane = threadIdx.x & 63, lr = lane & 15, g = lane >> 4;
  const int wave = threadIdx.x >> 6, nw = min((int)(blockDim.x >> 6), DM_NET_WAVES);
  const bool work = wave < nw;
  // inputs: row tile rt to Q (columns 0..31)
  if (work)
    for (int rt = wave; rt < DM_NET_RT; rt += nw)
      *(dm_bf16x8 DM_L*)(Q + (16 * rt + lr) * DM_NET_LDS_ROW + 8 * g) = input_fragment(A, S, row0 + 16 * rt + lr, g);
  __syncthreads();
  dm_f32x4 acc[DM_NET_RT][4];
  // layer 1 (K = 32): column block cb of every row tile, to P
  if (work)
    for (int cb = wave; cb < 4; cb += nw) {
#pragma unroll
      for (int rt = 0; rt < DM_NET_RT; ++rt) {
        const dm_bf16x8 a = lds_fragment(Q, 16 * rt + lr, 8 * g);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          acc[rt][ct] = dm_mfma_bf16(a, ld_bf16x8(W.w1 + (64 * cb + 16 * ct + lr) * DM_NET_KX + 8 * g),
                                     dm_f32x4{0.f, 0.f, 0.f, 0.f});
      }
      store_block(acc, W.b1, cb, P, lane);
    }
  __syncthreads();
  // layer 2 (K = 256): column block cb, from P to Q (the inputs are no longer needed)
  if (work)
    for (int cb = wave; cb < 4; cb += nw) {
#pragma unroll
      for (int rt = 0; rt < DM_NET_RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = dm_f32x4{0.f, 0.f, 0.f, 0.f};
      // two fragment sets in turn: the weights of step k + 32 are in flight while the
      // products of step k run (the scheduling barriers keep the loads ahead)
      const unsigned short DM_C* w2 = W.w2 + (64 * cb + lr) * DM_NET_HID + 8 * g;
      dm_bf16x8 b0[4], b1[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) b0[ct] = ld_bf16x8(w2 + 16 * ct * DM_NET_HID);
#pragma unroll 1
      for (int k0 = 0; k0 < DM_NET_HID; k0 += 64) {
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) b1[ct] = ld_bf16x8(w2 + 16 * ct * DM_NET_HID + k0 + 32);
        __builtin_amdgcn_sched_barrier(0);
        layer2_step(acc, b0, P, k0, lane);
        const int kn = k0 + 64 < DM_NET_HID ? k0 + 64 : k0;
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) b0[ct] = ld_bf16x8(w2 + 16 * ct * DM_NET_HID + kn);
        __builtin_amdgcn_sched_barrier(0);
        layer2_step(acc, b1, P, k0 + 32, lane);
      }
      store_block(acc, W.b2, cb, Q, lane);
    }
  __syncthreads();
  // layer 3 (N = 16, columns 0..2 real): row tile rt; lane (g, lr < 3) gets component lr of
  // rows 16 rt + 4g .. 16 rt + 4g + 3
  if (work)
    for (int rt = wave; rt < DM_NET_RT; rt += nw) {
      dm_f32x4 y = dm_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k0 = 0; k0 < DM_NET_HID; k0 += 32)
        y = dm_mfma_bf16(lds_fragment(Q, 16 * rt + lr, k0 + 8 * g), ld_bf16x8(W.w3 + lr * DM_NET_HID + k0 + 8 * g), y);
      if (lr < DM_NET_OUT) {
        const float bb = W.b3[lr];
        // the network predicts a whole backward-Euler step's correction; the Newton unknown of
        // a substep of adaptive halving, or the midpoint state of the implicit-midpoint rule,
        // takes its share: its Newton step over the whole time step
        const double sc = W.ystd[lr], share = dt / (A.midpoint ? 2.0 * A.dt : A.dt);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = row0 + 16 * rt + 4 * g + j;
          if (i < S.chain_nodes) {
            int c, k;
            system_row(D, S, i, c, k);
            const DmChain ch = D.chain[c];
            const float yv = y[j] + bb;
            put_guess(A, ch, k, lr, base_guess(A, dt, ch, k, lr) + share * sc * (double)yv, out);
          }
        }
      }
    }
  __syncthreads();               // Q is rewritten by the next block's inputs
}

// Step-start guess of system sid for the current warm mode (no-op for mode 0).  net: the
// network's LDS activations (two buffers of 16 DM_NET_RT rows).  out == null: written to the positions;
// else every row's displacement goes to out[row][3] and the positions stay.
__device__ __noinline__ void warm_guess(ArgsP Ap, int sid, unsigned short DM_L* net, double DM_G* out, double dt) {
  const DmStepArgs DM_C& A = *uniform(Ap);
  const DmDev DM_C& D = A.d;
  const DmSystem DM_C& S = D.sys[uniform(sid)];
  if (A.warm == 2) {
    for (int row0 = 0; row0 < S.chain_nodes; row0 += 16 * DM_NET_RT)
      network_block(A, dt, S, row0, net, net + 16 * DM_NET_RT * DM_NET_LDS_ROW, out);
  } else if (A.warm != 0) {
    for (int i = threadIdx.x; i < S.chain_nodes; i += blockDim.x) {
      int c, k;
      system_row(D, S, i, c, k);
      const DmChain ch = D.chain[c];
#pragma unroll
      for (int q = 0; q < 3; ++q) put_guess(A, ch, k, q, base_guess(A, dt, ch, k, q), out);
    }
  }
}
