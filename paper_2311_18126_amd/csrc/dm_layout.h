// dm_layout.h -- device data layout of the implicit DER step (shared by the host runtime
// and the kernels; not part of the public ABI).
//
// Terms used throughout:
//  system  : a connected set of rods (one rod, or rods joined at one shared end node).
//            One workgroup advances one system for all Newton iterations and steps.
//  chain   : one rod of a system in its stored node order.  Chain DOF r of node k is
//            4k + c (c = 0..2 position components, c = 3 the twist of edge k), so a bend/twist
//            stencil centred on node k occupies the 11 consecutive DOFs 4k-4 .. 4k+6 and the
//            chain Jacobian is banded with half-bandwidth 10.
//  border  : DOFs solved densely: for a single rod a 10-DOF separator in its middle; for a
//            joined system the shared node and, per rod, its joint-adjacent twist and node.
//  arm     : a contiguous run of chain DOFs eliminated by one wavefront in one direction,
//            ending next to the border (two arms per single rod, one per joined rod).
#pragma once

// The kernels' device pass sees the arrays the step writes in the global address space, the
// arrays it only reads (topology, parameters) in the constant one, and LDS pointers in the
// local one, so that loads and stores compile to global_/s_load/ds_ instructions instead of
// generic (flat) ones and read-only data need not be reloaded around stores; every other pass
// sees plain pointers of the same size and layout.
#if defined(__HIP_DEVICE_COMPILE__) && defined(DM_KERNEL_TU)
#define DM_G __attribute__((address_space(1)))
#define DM_L __attribute__((address_space(3)))
#define DM_C __attribute__((address_space(4)))
#else
#define DM_G
#define DM_L
#define DM_C
#endif

#define DM_HALF_BAND 10
#define DM_NDIAG 21          // band storage: row r holds columns r-10 .. r+10
#define DM_WIN 11            // elimination window (pivot + 10)
#define DM_FAC 12            // per eliminated row: 1/pivot, 10 upper entries, modified rhs
#define DM_FAC_STRIDE 16     // doubles per factor record (entries 12..15: write-only padding)
#define DM_MAX_CHAINS 8
#define DM_MAX_BORDER 40
#define DM_MAX_BSRC 8
#define DM_SEG 8             // terms per border term segment (padded with zero-pad terms)
#define DM_ST_G 8            // stencil gradient in (e_f, e_e, theta_f, theta_e)
#define DM_ST_H 64           // stencil Hessian in the same 8 variables, row-major
#define DM_ED 9              // edge: stretch gradient (3) + stiffness block (6, symmetric)
#define DM_ND 12             // node: residual (3) + Jacobian block (9, row-major)

struct DmChain {
  int n_nodes;     // nodes in this rod
  int node_tab;    // offset into chain_node (global node id of chain node k)
  int edge_tab;    // offset into chain_edge (global edge id of chain edge k)
  int st_off;      // global stencil id of the stencil centred on chain node 1
  int dof_off;     // offset of chain DOF 0 in the band / residual / delta arrays
  int b_lo, b_hi;  // border DOF range [b_lo, b_hi) in chain numbering
  int bmap_off;    // offset into bmap: border index of chain DOF b_lo + i
  int global_id;   // index of this chain in the chain array
  int rod;         // user rod id of this chain
};

struct DmArm {
  int chain;       // chain index (global)
  int dir;         // +1: eliminate chain DOFs first, first+1, ...; -1: first, first-1, ...
  int first;       // first chain DOF eliminated
  int count;       // DOFs eliminated; the next n_trail DOFs along dir are border DOFs
  int n_trail;     // trailing border DOFs in the elimination window (<= 10)
  int fac_off;     // offset (in records of DM_FAC_STRIDE doubles) of local row 0's record
};

// One term of a dense border entry: coef * (array kind)[idx], kinds 0 bpr, 1 st_H, 2 R,
// 3 st_g (the right-hand side column holds R and st_g terms), 4 the zero pad (padding of a
// segment: every segment holds DM_SEG terms).
struct DmBItem {
  int kind, idx;
  double coef;
};

struct DmSystem {
  int chain0, n_chains;
  int arm0, n_arms;
  int node0, n_nodes;    // global node range
  int edge0, n_edges;    // global edge range
  int st0, n_st;         // all stencils (chain stencils first, then joint stencils)
  int jst0, n_jst;       // joint stencils
  int nb;                // border size
  int bsrc_off;          // nb * DM_MAX_BSRC entries of (chain, dof) pairs, -1 terminated
  int bjst_off;          // n_jst * 11 border indices of joint-stencil local DOFs
  int bfix_off;          // nb fixed flags
  int chain_nodes;       // sum of chain node counts (band-assembly work items)
  int bent_off;          // nb (nb + 1) + 1 offsets into bent: entry b (nb + 1) + col sums the
                         // term segments bent[bent_off + e] .. bent[bent_off + e + 1] - 1
  int seg0, n_seg;       // the system's term segments (global segment indices)
  int seg_long;          // 1 if some entry has more than one segment
  int n_dof;             // sum of chain DOFs
};

// Device pointers.  All per-item arrays are structure-of-arrays.
struct DmDev {
  // topology
  const DmSystem DM_C* sys;
  const DmChain DM_C* chain;
  const DmArm DM_C* arm;
  const int DM_C* order;        // launch order of systems (largest first)
  const int DM_C* chain_node;
  const int DM_C* chain_edge;
  const int DM_C* bmap;
  const int DM_C* bsrc;         // pairs (chain global index, chain DOF)
  const int DM_C* bjst;
  const int DM_C* bent;         // border entry -> first term segment (per system from bent_off)
  const DmBItem DM_C* bitem;    // border entry terms in segments of DM_SEG, in entry order
  const int DM_C* bsch;         // [arms][110]: where each Schur slot of an arm adds into the
                                // border, (row << 16) | (col << 8) | slot, or -1 (none or clamped)
  const unsigned char DM_C* bfix;
  const unsigned char DM_C* cfix;   // per chain DOF: 1 if clamped
  const unsigned DM_C* nmask;   // [chain-node rows][4]: clamped and border bits of chain DOFs
                                // 4k-12 .. 4k+19 (bit i: DOF 4k-12+i), owner flag, padding
  // nodes
  const double DM_C* mass;
  const double DM_C* radius;
  const double DM_C* force;     // [3][n_nodes]
  const int DM_C* node_owner;   // chain that assembles the node's own terms
  const int DM_C* node_home;    // [3][n_nodes]: delta index (>= 0) or -1 - border index
  // edges
  const int DM_C* en;           // [2][n_edges] tail, head
  const double DM_C* ebar;
  const double DM_C* arc0;      // rest arclength of the edge's rod at its first node
  // self-contact (dm_set_self_contact): per system a dense n x n Newton matrix over its chain
  // DOFs and n doubles after it, at sc_off[system] doubles into sc_mat
  double DM_G* sc_mat;
  const long long DM_C* sc_off;
  const double DM_C* EA;
  const double DM_C* Ith;
  const double DM_C* moment;
  const int DM_C* edge_home;
  // stencils
  const int DM_C* sn;           // [3][n_st] previous, centre, next node
  const int DM_C* se;           // [2][n_st] edge f, edge e
  const int DM_C* ssign;        // bit 0: edge f stored reversed, bit 1: edge e stored reversed
  const double DM_C* Vbar;
  const double DM_C* kbend;     // EI / Vbar
  const double DM_C* ktwist;    // GJ / Vbar
  const double DM_C* kbar;      // [2][n_st] static integrated natural curvature
  const double DM_C* tbar;
  const double DM_C* act;       // [3][n_st] A (1/m), f, phi; A is NaN when not actuated
  // warm-start network inputs per chain-node row (rows: chains in order, nodes in chain order)
  const double DM_C* nconst;    // [rows][3] log10 E, radius, mean rest length of the node's edges
  // state
  double DM_G* x;  double DM_G* x0;  double DM_G* v;      // [3][n_nodes]
  double DM_G* vprev;                           // [3][n_nodes] velocity before the last step
  double DM_G* vprev2;                          // [3][n_nodes] velocity before the one before
  double DM_G* th; double DM_G* th0; double DM_G* om;     // [n_edges]
  double DM_G* tref; double DM_G* d1ref;             // [3][n_edges]
  double DM_G* bref;                            // [n_st]
  double DM_G* time;                            // [n_systems]
  // scratch
  double DM_G* st_g;   // [8][n_st]
  double DM_G* st_H;   // [64][n_st]
  double DM_G* ed;     // [9][n_edges]
  double DM_G* nd;     // [12][n_nodes]
  double DM_G* band;   // [n_dof_total][21]
  double DM_G* bpr;    // [bmap entries][21]: border-column part of each chain's border rows
  double DM_G* R;      // [n_dof_total]
  double DM_G* fac;    // [n_dof_total][12]
  double DM_G* delta;  // [n_dof_total]
  double DM_G* babs;   // [bmap entries]: sum_k |J_rk| s_k over the band columns of a border row r
                       // (the part of its rounding-floor row sum held by one chain)
  double DM_G* zpad;   // [16] zeros, never written: where out-of-range solver loads are sent
  // statistics
  int DM_G* s_steps; int DM_G* s_iters; int DM_G* s_status; double DM_G* s_res; int DM_G* s_floor;
  int DM_G* s_fallback;  // warm-started attempts that had to restart from the step start
  int DM_G* s_halved;    // substeps whose failed Newton solve was redone as two halves
  double DM_G* s_floor_res;  // largest residual among (sub)steps ended at the rounding floor
  double DM_G* s_floor_est;  // the floor estimate of that (sub)step
  double DM_G* dbg;     // [n_systems][8] phase timers in diagnosis builds; null otherwise
  int n_nodes_tot, n_edges_tot, n_st_tot;
};

// Warm-start network of the step kernel, 26 -> 256 -> 256 -> 3 with ReLU: bfloat16 bit
// patterns of W1 [256][32], W2 [256][256] and W3 [16][256] (zero padded, reduction index
// contiguous), float32 biases, and the float64 input standardisation and output scales.
#define DM_NET_IN 26
#define DM_NET_HID 256
#define DM_NET_OUT 3
#define DM_NET_KX 32          // input width padded to one matrix-core reduction step
#define DM_NET_OUTP 16        // output width padded to one matrix-core tile
#define DM_NET_WAVES 4        // wavefronts of a workgroup that run the network
#define DM_NET_LDS_ROW 264    // bfloat16 per activation row in LDS (256 + 8 padding)
#define DM_NET_RT 3           // 16-row tiles per network block of the step kernel
#define DM_NET_LDS_BYTES (2 * 16 * DM_NET_RT * DM_NET_LDS_ROW * 2)   // two activation buffers
struct DmNetView {
  const unsigned short DM_C* w1; const unsigned short DM_C* w2; const unsigned short DM_C* w3;
  const float DM_C* b1; const float DM_C* b2; const float DM_C* b3;
  const double DM_C* mean; const double DM_C* sd; const double DM_C* ystd;
};

struct DmStepArgs {
  DmDev d;
  DmNetView net;
  double dt, tol;      // dt: the Newton solve's step (half the time step under midpoint)
  double floor_factor; // rounding-floor estimate factor * eps * || |J| s ||_2 (0: no floor rule)
  double g[3];
  double damping;
  double floor_z, delta, nu, mu, kc;
  int floor_on;
  int max_iter, nsteps, line_search;
  int warm;        // step-start guess: 0 none (x_n), 1 x_n + dt v_n, 3 + dt a_n, 4 + dt (a_n + j_n),
                   // 2 mode 4 plus the network's correction; a failed guess restarts from x_n
  int warm_max_iter;   // Newton iterations allowed to the warm-started attempt
  int accum;       // 1: add to the statistics (one-step launches) and skip systems that failed
  int net_lds;     // byte offset of the network's LDS activations (warm == 2)
  int midpoint;    // 1: implicit midpoint; dt is then half the time step (the Newton solve is
                   // backward Euler to the midpoint) and the commit extrapolates to the step end
  int max_halvings;  // adaptive time stepping: a failed (sub)step is redone as two halves, at
                     // most this many levels deep (0: off)
  const int DM_C* skip;   // [n_systems] nonzero: the system takes no step in this launch (or null)
  int n_systems;
  int max_nb, max_arms;
  int max_seg;     // largest number of border term segments of a system (LDS partial sums)
  // edge-edge self-contact of single-rod systems (off: sc_on = 0)
  int sc_on, sc_cap, sc_max_edges, sc_lds, sc_pb;   // pair slots per system (a power of two), LDS offset
  double sc_delta, sc_kc, sc_mu, sc_nu;
};

// Discrete adjoint of a stored trajectory segment (single-rod systems without contact).
// A stored state holds, at offsets in doubles: x [3][NN] at 0, v [3][NN] at 3NN,
// theta [NE] at 6NN, omega [NE] at 6NN+NE, t_ref [3][NE] at 6NN+2NE, d1_ref [3][NE] at
// 6NN+5NE, beta_ref [NS] at 6NN+8NE, time [n_systems] at 6NN+8NE+NS.
struct DmAdjDev {
  const double DM_C* seg;       // states 0 .. seg_len of the segment, `stride` doubles apart
  const double DM_C* dLdtip;    // [n_steps][n_rods][3]: loss gradient w.r.t. the tip after step g+1
  double DM_G* ax;  double DM_G* av;      // [3][NN] cotangents of x, v
  double DM_G* ath; double DM_G* aom;     // [NE] cotangents of theta, omega
  double DM_G* atref; double DM_G* ad1;   // [3][NE] cotangents of t_ref, d1_ref
  double DM_G* akap;                      // [2][NS] accumulated gradient w.r.t. integrated kbar
  double DM_G* lam;                       // [3][NN] then [NE]: the adjoint solution lambda
  double DM_G* pst;                       // [16][NS] per-stencil parameter derivatives
  double DM_G* pe;                        // [3][NE] per-edge cotangent of the edge vector
  long long stride;
  int seg_len, step0, n_rods;
};

struct DmAdjArgs {
  DmStepArgs s;                 // first member: the step arguments at offset 0
  DmAdjDev a;
};

// Gradient of a weighted sum of stencil curvatures of an equilibrium (dm_curvature_adjoint_kernel).
struct DmCurvAdj {
  const double DM_C* wst;   // [n_st] weight of each stencil's kappa_1 (zero: not in the sum)
  double DM_G* mu;          // [3 NN + NE] solution of J mu = d(sum w kappa1)/dq
  double DM_G* pst;         // [n_st] derivative with respect to the stencil's natural curvature (1/m)
  const int DM_C* skip;     // [n_systems] nonzero: the system is left alone (or null)
};

struct DmCurvArgs {
  DmStepArgs s;             // first member: the step arguments at offset 0
  DmCurvAdj c;
};

struct dm_mlp;
// Device operands of a network for the step kernel (host function of dm_mlp.hip).
void dm_mlp_view(const dm_mlp* m, DmNetView* v);
