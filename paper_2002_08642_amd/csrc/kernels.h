// kernels.h - device kernels of the penalized pseudo-spectral step (gfx950).
//
// Data layout in HBM (C order, x fastest):
//   compact spectrum  [iz][iy][ix]        ix in [0, Kx], iy, iz in the 2/3 band
//   z-pass output     [z][iy][ix]         (band in y and x, all z)
//   y-pass output     [z][y][ix]          (band in x, all y and z)
//   physical          [z][y][x]
// The ix axis of the spectral layouts is padded to a pitch kxp of whole
// 128-byte lines, so that every row segment a workgroup moves is line aligned.
// The step is five passes over these layouts (z-inverse + curl, y-inverse,
// fused x pass, y-forward, z-forward + projection + update) plus the mask
// kernels and the reduction that also produces the adaptive dt.
#pragma once

#include "fft_lds.h"

namespace fsi {

constexpr int kNT = 256;  // threads per workgroup of the mask and reduction kernels

enum ColMode {
  COL_INV_PLAIN = 0,
  COL_INV_CURL = 1,
  COL_FWD_PLAIN = 2,
  COL_FWD_PROJECT = 3,
  COL_FWD_UPDATE = 4,
  COL_FWD_ACC = 5,       // adjoint: out[f] += m_k * forward(in[f])   (m_k = 1 at kx = 0, else 2)
  COL_FWD_ACC_CURL = 6,  // adjoint: out += m_k * (i k x forward(in[0..2]))
  COL_INV_CURL5 = 7,     // z inverse of u and of omega_x, omega_y (5 outputs)
  COL_INV_WZ = 8,        // y inverse of 5 fields plus omega_z = i (kx uy - ky ux) (6 outputs)
  COL_FWD_UPDATE_Z = 9,  // COL_FWD_UPDATE, then COL_INV_CURL5 of the new velocity into zout
  COL_FWD_SPONGE = 10,   // sponge term -(1/C_sp) i k x forward(in[0..2]) / |k|^2 into out (compact)
  COL_ADJ_MU = 11        // adjoint: update/projection transpose on (uh = lambda_u, nh = lambda_N)
                         // in place, then z inverse of mu = P(lambda_N)/(m_k N^3) into out (3 fields);
                         // with spadj also the sponge cotangent nu of mu (compact)
};
enum XMode { X_FUSED = 0, X_C2R = 1, X_R2C = 2 };

// Device scalars shared by the passes of one step.
struct DevScalars {
  double dt[2];     // dt_n and dt_{n-1}, indexed by step parity
  double t;         // time after the last completed step
  double info[8];   // F[3], E, umax, dt, nonfinite flag, spare
  double fst[3];    // force of the static penalization (weighted)
};

template <typename T>
struct ColArgs {
  const cpx<T>* in;
  cpx<T>* out;
  long long in_fs, out_fs;  // field strides (complex elements)
  long long in_bs, out_bs;  // slice strides (blockIdx.y)
  int C;                    // columns per slice
  int ld;                   // row pitch of in and out (complex elements)
  int n;                    // transform length
  int K;                    // band half width along the transform axis
  int nf;                   // fields (plain modes)
  FftPlan plan;
  const cpx<T>* tw;
  // spectral bookkeeping: column c = iy * kxp + ix, valid while ix < kx1
  // (kxp pads the x band to whole 128-byte lines)
  int kx1;
  int kxp;
  int Ky;
  T kfx, kfy, kfz;  // 2 pi / L per axis
  T scale;          // factor applied to forward outputs
  // projection / update (z-forward pass)
  cpx<T>* uh;
  cpx<T>* nh;
  long long cfs;  // compact field stride
  const DevScalars* sc;
  int cur;    // parity index of dt_n
  int first;  // 1: integrating-factor Euler step
  T nu;
  cpx<T>* pi;  // update pass: total pressure Pi_hat = -i k.N'/|k|^2 (compact), NULL = not kept
  cpx<T>* zout;       // COL_FWD_UPDATE_Z: the five z-inverse fields of the new velocity
  long long zout_fs;  // their field stride (row pitch ld, as the input)
  const cpx<T>* tsp;  // update passes: sponge term added before the projection, NULL = none
  T csp_inv;          // COL_FWD_SPONGE: 1 / C_sp
  // COL_ADJ_MU (uh, nh: the cotangents of u_hat and of the previous nonlinear
  // term; first, nu, cfs as for the update)
  double adt, adtp;      // dt of the reversed step and the one before
  double invN3;          // 1 / (nx ny nz)
  const cpx<T>* lpi;     // pressure seed (normalized R2C of the cotangent of Pi), NULL = none
  cpx<T>* spadj;         // sponge on: nu = -(1/C_sp) i k x mu / |k|^2 (compact; csp_inv), NULL = none
};

// Sponge mask on the physical grid: phys[f] *= max(gx[x], gy[y], gz[z]), f < 3.
template <typename T>
struct SpongeArgs {
  T* phys;
  long long npts;
  int nx, ny;
  const T* g;  // gx (nx values), then gy (ny), then gz (nz)
  int nz;
};

template <typename T>
struct XArgs {
  cpx<T>* spec;       // [f][line][ld], kx1 valid entries per line
  cpx<T>* gout;       // fused mode: G out [3][line][ld] (stride sfs; may be spec)
  long long sfs;      // field stride of spec
  int ld;             // line pitch of spec (>= kx1, whole 128-byte lines)
  T* phys;            // [f][line][n] (plain modes)
  long long pfs;
  int nlines;         // ny * nz
  int ny;
  int n;              // nx
  int kx1;            // Kx + 1
  FftPlan plan;
  const cpx<T>* tw;
  // mask sub-box (fused mode); bnx == 0 means no wing
  const T* chi;
  const T* us;        // [3][cell]
  int bx0, by0, bz0, bnx, bny, bnz;
  long long bcells;
  T inv_eta;
  double* partials;   // [gridDim.x][8]
  // velocity kept on the pressure box (FSI mode), [3][cell]; pnx = 0: off
  T* up;
  int px0, py0, pz0, pnx, pny, pnz;
  long long pcells;
  // static z-independent penalization (fused mode; NULL: off): chi [y][x],
  // u_s [3][y][x] (component stride ny * nx), force weight [y][x]
  const T* st_chi;
  const T* st_us;
  const T* st_w;
};

// p = Pi - |u|^2/2 at the cells of the pressure box (out, FP64), and the
// embedding of box values into a full grid field.
template <typename T>
struct BoxArgs {
  const T* pi;    // full grid [z][y][x] (pbox_pressure) / out grid (embed)
  const T* up;    // [3][cell]
  int nx, ny, nz;
  int px0, py0, pz0, pnx, pny, pnz;
  long long pcells;
  double* out;       // [cell] (pbox_pressure)
  const T* in;       // [cell] (embed)
  T* grid;           // full grid (embed)
};

// Sampling of p = Pi - |u|^2 / 2 with the 4-point delta kernel: Pi on the full
// grid ([z][y][x]), u on the pressure box, points in FP64.
template <typename T>
struct PressArgs {
  const T* pi;
  const T* up;
  int nx, ny, nz;
  int px0, py0, pz0, pnx, pny, pnz;
  long long pcells;
  const double* pts;  // [ns][3]
  int ns;
  double dx, dy, dz;
  double* out;        // [ns]
};

// The mask geometry is evaluated in FP64 in both precisions (it is a small
// part of the step); chi and u_s are stored in the bulk precision.
template <typename T>
struct MaskArgs {
  const double* x;     // [nv][3]
  const double* v;     // [nv][3]
  const int* tri;      // [nt][3]
  int nt;
  unsigned long long* key1;  // [cell] (truncated FP32 distance bits << 32) | triangle
  unsigned long long* key2;  // [cell] (low FP64 mantissa bits << 32) | triangle
  T* chi;
  T* us;               // [3][cell]
  int bx0, by0, bz0, bnx, bny, bnz;
  long long bcells;
  double dx, dy, dz;
  double rsup;         // support radius
  double tw, h;
  int profile;
  // grid output (launch_mask_grid only): chi and u_s written to full grids
  // [nz][ny][nx] (u_s component stride gcells) instead of the sub-box arrays
  int gnx, gny;
  long long gcells;
};

// ---------------------------------------------------------------------------
// adjoint of one step (dt held fixed)
// ---------------------------------------------------------------------------

// The spectral part of the reverse step (per compact mode) is the column pass
// COL_ADJ_MU (ColArgs above).

// Fused x pass of the reverse step: C2R of u, omega and lambda_G (9 fields),
// lambda_u = omega x lambda_G - (chi/eta) lambda_G + (dV/eta) chi g,
// lambda_omega = lambda_G x u, and the mask cotangents
// lambda_chi = (g dV - lambda_G).(u - u_s)/eta, lambda_us = chi (lambda_G - g dV)/eta;
// R2C of lambda_u, lambda_omega (6 fields).
template <typename T>
struct XAdjArgs {
  cpx<T>* spec;  // [9][line][ld] in, [6][line][ld] out
  // u, omega of the step from its tape (fields 0-5, stride sfs); NULL: fields
  // 0-5 of spec
  const cpx<T>* utape;
  long long sfs;
  int ld;
  int nlines, ny, n, kx1;
  FftPlan plan;
  const cpx<T>* tw;
  const T* chi;
  const T* us;
  T* lchi;       // [cell] out
  T* lus;        // [3][cell] out
  int bx0, by0, bz0, bnx, bny, bnz;
  long long bcells;
  T inv_eta;
  T g0, g1, g2;  // dV * dJ/dF
  // pressure seed (FSI coupling): cotangent of p = Pi - |u|^2/2 on the pressure
  // box, adds -u lp to lambda_u there (pnx = 0: none)
  const T* lp;
  int px0, py0, pz0, pnx, pny, pnz;
  long long pcells;
};

// Mask adjoint: per triangle, sums over the cells it wins of the cotangents of
// its vertex positions and velocities (through the distance, the profile and
// the barycentric weights of the closest point).
template <typename T>
struct MaskAdjArgs {
  const double* x;
  const double* v;
  const int* tri;
  int nt;
  const unsigned long long* key2;
  const T* chi;
  const T* lchi;
  const T* lus;
  int bx0, by0, bz0, bnx, bny, bnz;
  long long bcells;
  double dx, dy, dz;
  double rsup, tw, h;
  int profile;
  double* tgrad;  // [nt][18]: d/dx of (a, b, c), then d/dv of (a, b, c)
};

struct FinalArgs {
  const double* partials;
  int np;
  DevScalars* sc;
  int cur;        // parity index where dt_n is written
  int adaptive;   // 0: dt_n = dt_fixed
  double dt_fixed;
  double cfl_dx;  // cfl * dx_min
  double cap;     // min(c_eta * eta, dt_max)
  double dV;
  double inv_eta;
};

}  // namespace fsi
