// Kernel argument structures and host-side launch wrappers.
#pragma once
#include "layout.hpp"

namespace psfd {

enum LoadOp { LD_PLAIN = 0, LD_VX = 1, LD_INJECT = 2, LD_VXE = 3, LD_INJECT_T = 4, LD_UPD_VX = 5, LD_UPD_SLOT = 6 };

struct GState;
// The Givens step of the previous Arnoldi step, left to an apply kernel of
// this one: an extra block of the kernel runs it (see givens_task), and the
// other blocks take the scale of the step's input vector from the same norm
// partials (nblk per instance in part, instance stride nblk) instead of in_scale.
// The kernel's blocks must have at least GIVENS_THREADS threads.
struct GivensTask {
  GState* st;
  int* run;
  const double2* part;
  int nblk;
  int by_pend;  // 1: only the instances with a pending update (GState::pend) take the task
                // and the scale; the others' input was scaled on load
};
// The Gram-Schmidt update of column j - 1, left to the forward square-plane
// kernel of step j (LD_UPD_VX, lock-step solves): every plane block sums the
// projection partials of the step before (dpart, DotBlocks<float2> per value,
// PSTR values per instance), forms slot_j -= sum_{i<j} h_i s_i slot_i over its
// plane, stores it, and leaves the plane's ||slot_j||^2 in part[b * planes + plane];
// the block of plane 0 stores h and ||w||^2 before the update for the Givens step.
// The vector enters the transform unscaled: the next kernel applies its scale.
// LD_UPD_VX: j >= 1, every instance at step j. LD_UPD_SLOT: per instance, j = 0
// (the first step of a cycle: no update, slot 0 scaled on load by S.inv_norm, as
// LD_VX does) or j < 0 (instances at different steps: from its state; with a
// pending update (pend) the update of column S.j on slot S.j + 1, else slot S.j
// scaled on load). Both run the same arithmetic for the same case.
struct UpdateTask {
  const void* V;        // basis of instance 0; slot i of instance b at V + b bsv + i ldv
  long long ldv, bsv;
  GState* st;
  const double2* dpart;
  double2* part;
  int j;
};
// The Gram-Schmidt projections of the new Arnoldi vector, left to the kernel
// that writes it (ST_DOTS, inverse square planes): each plane block also forms
// the partial dot products <slot_i, w> (i = 0..j) and ||w||^2 over its plane
// and stores them where the projection pass would (PSTR values per instance,
// DotBlocks<float2> partials each: the plane's own, zeros in the others).
struct DotTask {
  const void* V;        // basis of instance 0; slot i of instance b at V + b bsv + i ldv
  long long ldv, bsv;
  GState* st;           // j of each instance when jh < 0; pend is set (the update of the
                        // column is pending)
  double2* part;
  int jh;               // >= 0: every running instance stands at step jh
};
enum StoreOp { ST_PLAIN = 0, ST_AXPBY = 1, ST_DOTS = 2 };

// One launch of the transverse (x/y) FFT kernel over tiles of every plane of
// every instance. A tile is ty rows x tx columns of one (component, z) plane.
struct TileArgs {
  int nx, ny, nz, log2nx, log2ny;
  int tx, ty, pitch;
  int tiles_x, tiles_y;
  int do_x, do_y;
  VecRef in, aux, out;   // fields [3][nz][ny][nx]
  VecRef vol;            // contrast delta_eps [nz][ny][nx] (times k0^2 on load)
  const double* tab;     // per-instance tables (TabLayout), stride tab_stride doubles
  long long tab_stride;
  const double2* eup;    // LD_INJECT: upgoing amplitudes [ny*nx][3] per instance
  long long eup_stride;  //   (LD_INJECT_T: eup = b_dn, eup2 = b_up, see launch_adjoint_source)
  const double2* eup2;
  const void* tw;        // twiddle table in the working precision
  double alpha, gamma;   // ST_AXPBY: out = alpha * aux + gamma * result
  const int* active;     // optional per-instance flags (0 = skip)
  const double* in_scale;  // LD_VX, optional: in scaled by in_scale[b * scale_stride] on load (in is not modified)
  long long scale_stride;
  GivensTask gv;           // LD_VX square planes, optional (gv.st null: none)
  DotTask dt;              // ST_DOTS
  UpdateTask up;           // LD_UPD_VX
};

// One launch of the z-pencil kernel: forward z-FFT over the zero-padded
// length pz = 2 nz, multiply by the dyadic kernel, inverse z-FFT, keep nz.
struct PencilArgs {
  int nx, ny, nz, pz, log2pz, bx, pitch, nblk_x;
  VecRef w;
  const double* tab;
  long long tab_stride;
  const void* tw;
  int transpose;         // use the kernel at the negated wavevector (bilinear transpose)
  int reflect;           // add the layered-stack response R_vol T_R K_top (monolithic coupling)
  const int* active;
  GivensTask gv;         // optional (gv.st null: none): the pending Givens step in one extra
                         // block; the other blocks scale the input by the new vector's scale
  int yq;                // w in the quarter-plane layout of launch_qplane (nblk_x = nx / 4)
};

struct TileShape { int tx, ty, do_x, do_y, nthr; size_t lds; int pitch; };

// Byte offsets of a pencil block's LDS regions: the data [pz][3 bx], the phase
// factors [Q + nz / Q][bx] of the stack response (Q = min(8, nz)) and the window
// factors [pz / 2 + 1][bx], in elements of esz bytes; then, 16-byte aligned,
// E_up [bx][3], the readout partial sums [nthr] and the order constants [bx][7]
// (16-byte words), and the twiddles [pz] (esz).
struct PencilLds {
  int fac, win, eup, part, ptab, twl, total;
  __host__ __device__ PencilLds(int pz, int bx, int nthr, int esz) {
    const int nz = pz / 2, q = nz < 8 ? nz : 8;
    fac = pz * 3 * bx * esz;
    win = fac + bx * (q + nz / q) * esz;
    eup = (win + bx * (pz / 2 + 1) * esz + 15) / 16 * 16;
    part = eup + 3 * bx * 16;
    ptab = part + nthr * 16;
    twl = ptab + 7 * bx * 16;
    total = twl + pz * esz;
  }
};

template <class T, bool INV, int LD, int ST>
void launch_tile(const TileArgs& a, int nplanes, int nbatch, int nthr, size_t lds, hipStream_t s);
// whether launch_tile runs the square-plane kernel for these arguments (the
// kernel that can carry a GivensTask)
bool tile_is_plane(const TileArgs& a, size_t esz);
// whether launch_tile can store with ST_DOTS for these arguments (FP32 64 x 64 and
// 128 x 128 planes, at most DotBlocks<float2> planes per instance)
bool tile_takes_dots(const TileArgs& a, size_t esz);
// whether launch_tile can load with LD_UPD_VX / LD_UPD_SLOT for these arguments (FP32 64 x 64 and
// 128 x 128 planes)
bool tile_takes_update(const TileArgs& a, size_t esz);
template <class T>
void launch_pencil(const PencilArgs& a, int nbatch, int nthr, size_t lds, hipStream_t s);
// Quarter-plane transverse kernels of the operator apply on 128 x 128 planes
// (and 256 x 256 in FP32): forward (LD_VX, ST_PLAIN) into the quarter-plane layout, inverse
// (LD_PLAIN, ST_PLAIN or ST_AXPBY) from it; nplanes = 3 nz, no GivensTask.
// The pencil between them runs with PencilArgs::yq.
template <class T, bool INV, int LD, int ST>
void launch_qplane(const TileArgs& a, int nplanes, int nbatch, hipStream_t s);
// whether a shape (and its pencil's columns bx and threads) takes them: 128 x 128
// planes, and 256 x 256 in FP32 (esz 8)
bool qplane_shape(int nx, int ny, int nz, int pz, int bx, int nthr, size_t esz);

// per-order readouts of the source density spectra (FP64):
// adn = (i dz / 2 beta) P- sum_k exp(i beta z_k) f_q(z_k) / (NxNy), aup likewise at z = T.
void launch_readout(int nx, int ny, int nz, VecRef spec, const double* tab, long long tab_stride,
                    double2* adn, double2* aup, long long ostride, const int* active, int nbatch, hipStream_t s);
// eup <- T_R (adn + e_inc), with partial sums of |change|^2 and |new|^2 per block
void launch_reflect(int nx, int ny, const double* tab, long long tab_stride, const double2* adn,
                    double2* eup, long long ostride, double* part, int nblk, const int* active, int nbatch,
                    hipStream_t s);
// Adjoint source per order from the cotangent G = dL/dRe a + i dL/dIm a of the
// orders, with c = conj(G):
// b_dn = (i dz / 2 beta)(1/NxNy) P- T_R^T (exp(i beta T) c), b_up = (i dz / 2 beta)(1/NxNy) P+ c
void launch_adjoint_source(int nx, int ny, const double* tab, long long tab_stride, const double2* g,
                           double2* bdn, double2* bup, long long ostride, int nbatch, hipStream_t s);
// grad = conj(k0^2 sum_c lam_c u_c) per voxel (complex128 [nz][ny][nx]), the
// gradient dL/dRe + i dL/dIm of the loss whose cotangent made the adjoint source
void launch_gradient(long long N, const double* tab, long long tab_stride, const double2* lam, const double2* u,
                     long long n3stride, double2* grad, long long gstride, int nbatch, hipStream_t s);
// per-order part of an instance table (beta, exp(i beta L), keep, T_R) from kx, ky,
// the scalars in tab and the stack lay[0..nl+1] = ambient, layers, substrate
void launch_stack_table(int nx, int ny, double* tab, const double4* lay, int nl, double k0sq, double phi,
                        hipStream_t s);
// orders = eup exp(i beta T) + aup
void launch_orders(int nx, int ny, const double* tab, long long tab_stride, const double2* eup,
                   const double2* aup, double2* orders, long long ostride, int nbatch, hipStream_t s);

}  // namespace psfd
