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

#define DM_HALF_BAND 10
#define DM_NDIAG 21          // band storage: row r holds columns r-10 .. r+10
#define DM_WIN 11            // elimination window (pivot + 10)
#define DM_FAC 12            // per eliminated row: 1/pivot, 10 upper entries, modified rhs
#define DM_MAX_CHAINS 8
#define DM_MAX_BORDER 40
#define DM_MAX_BSRC 8
#define DM_ST_G 11           // stencil gradient entries (local DOFs)
#define DM_ST_H 66           // stencil Hessian upper triangle (11 x 11)
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
};

struct DmArm {
  int chain;       // chain index (global)
  int dir;         // +1: eliminate chain DOFs first, first+1, ...; -1: first, first-1, ...
  int first;       // first chain DOF eliminated
  int count;       // DOFs eliminated; the next n_trail DOFs along dir are border DOFs
  int n_trail;     // trailing border DOFs in the elimination window (<= 10)
  int fac_off;     // offset (in DM_FAC records) of local row 0's factor record
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
  int n_dof;             // sum of chain DOFs
};

// Device pointers.  All per-item arrays are structure-of-arrays.
struct DmDev {
  // topology
  const DmSystem* sys;
  const DmChain* chain;
  const DmArm* arm;
  const int* order;        // launch order of systems (largest first)
  const int* chain_node;
  const int* chain_edge;
  const int* bmap;
  const int* bsrc;         // pairs (chain global index, chain DOF)
  const int* bjst;
  const unsigned char* bfix;
  const unsigned char* cfix;   // per chain DOF: 1 if clamped
  // nodes
  const double* mass;
  const double* radius;
  const double* force;     // [3][n_nodes]
  const int* node_owner;   // chain that assembles the node's own terms
  const int* node_home;    // [3][n_nodes]: delta index (>= 0) or -1 - border index
  // edges
  const int* en;           // [2][n_edges] tail, head
  const double* ebar;
  const double* EA;
  const double* Ith;
  const double* moment;
  const int* edge_home;
  // stencils
  const int* sn;           // [3][n_st] previous, centre, next node
  const int* se;           // [2][n_st] edge f, edge e
  const int* ssign;        // bit 0: edge f stored reversed, bit 1: edge e stored reversed
  const double* Vbar;
  const double* kbend;     // EI / Vbar
  const double* ktwist;    // GJ / Vbar
  const double* kbar;      // [2][n_st] static integrated natural curvature
  const double* tbar;
  const double* act;       // [3][n_st] A (1/m), f, phi; A is NaN when not actuated
  // state
  double* x;  double* x0;  double* v;      // [3][n_nodes]
  double* th; double* th0; double* om;     // [n_edges]
  double* tref; double* d1ref;             // [3][n_edges]
  double* bref;                            // [n_st]
  double* time;                            // [n_systems]
  // scratch
  double* st_g;   // [11][n_st]
  double* st_H;   // [66][n_st]
  double* ed;     // [9][n_edges]
  double* nd;     // [12][n_nodes]
  double* band;   // [n_dof_total][21]
  double* R;      // [n_dof_total]
  double* fac;    // [n_dof_total][12]
  double* delta;  // [n_dof_total]
  // statistics
  int* s_steps; int* s_iters; int* s_status; double* s_res; int* s_floor;
  int n_nodes_tot, n_edges_tot, n_st_tot;
};

struct DmStepArgs {
  DmDev d;
  double dt, tol, stag_tol;
  double g[3];
  double damping;
  double floor_z, delta, nu, mu, kc;
  int floor_on;
  int max_iter, nsteps, line_search;
  int n_systems;
  int max_nb, max_arms;
};
