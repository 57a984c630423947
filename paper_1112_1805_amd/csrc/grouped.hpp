// Grouped launches for batches of images of different sizes and label counts.
//
// One ADMM iteration of an image is a fixed sequence of kernels (adjoint column pass, row
// pass back to real rows, pixel step, forward row and column passes, synthesis column pass,
// the fused row pass).  In a batch, each step of that sequence is issued once for all
// images whose kernel has the same compile-time configuration: the launch's blocks are the
// images' grids laid end to end, a table gives every block its image (task), and the task
// holds that image's parameters.  Every block then runs exactly the code and arithmetic of
// the single-image kernel, so a batch solve equals the images' separate solves bit for bit,
// while each launch fills the whole GPU instead of one image's share of it.
#pragma once
#include "kernels.hpp"
#include "generic.hpp"

namespace shs {

// One image's part of a grouped launch: its kernel parameters and its own grid (gx x gy
// blocks, flattened x-fastest), starting at block `start` of the launch.
template <class P>
struct GroupTask {
  P p;
  GenParams gp;   // mixed-radix plan (unused by the power-of-two kernels)
  int gx, gy, start, pad;
};

// The task of this block (bt: task index per launch block) and the block's coordinates in
// that task's grid.
template <class P>
__device__ __forceinline__ const GroupTask<P>& group_task(const GroupTask<P>* __restrict__ tasks,
                                                         const uint16_t* __restrict__ bt) {
  return tasks[__builtin_amdgcn_readfirstlane(int(bt[blockIdx.x]))];
}
template <class P>
__device__ __forceinline__ BlockId group_block(const GroupTask<P>& T) {
  const int local = int(blockIdx.x) - T.start;
  return BlockId{local % T.gx, local / T.gx, T.gx};
}

// ---- power-of-two sizes (compile-time N)
template <int N, int MODE, int ST, bool STATS>
__global__ __launch_bounds__(RowGeom<N>::THREADS) void kg_row(const GroupTask<RowParams>* __restrict__ tasks,
                                                              const uint16_t* __restrict__ bt) {
  const GroupTask<RowParams>& T = group_task(tasks, bt);
  row_body<N, MODE, ST, STATS>(T.p, group_block(T));
}
template <int N>
__global__ __launch_bounds__(ColCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(3))) void kg_col_fwd(
    const GroupTask<ColParams>* __restrict__ tasks, const uint16_t* __restrict__ bt) {
  const GroupTask<ColParams>& T = group_task(tasks, bt);
  col_fwd_body<N>(T.p, group_block(T));
}
template <int N>
__global__ __launch_bounds__(ColCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(ColGeom<N>::WPE))) void kg_col_syn(
    const GroupTask<ColParams>* __restrict__ tasks, const uint16_t* __restrict__ bt) {
  const GroupTask<ColParams>& T = group_task(tasks, bt);
  col_syn_body<N>(T.p, group_block(T));
}
template <int N>
__global__ __launch_bounds__(ColCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(ColGeom<N>::WPE))) void kg_col_ana(
    const GroupTask<ColParams>* __restrict__ tasks, const uint16_t* __restrict__ bt) {
  const GroupTask<ColParams>& T = group_task(tasks, bt);
  col_ana_body<N>(T.p, group_block(T));
}
template <int N>
__global__ __launch_bounds__(ColCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(3))) void kg_col_final(
    const GroupTask<ColParams>* __restrict__ tasks, const uint16_t* __restrict__ bt) {
  const GroupTask<ColParams>& T = group_task(tasks, bt);
  col_final_body<N>(T.p, group_block(T));
}

// ---- mixed-radix sizes (runtime N; dynamic LDS sized for the group's largest image)
template <int MODE, int ST, bool STATS, int RW>
__global__ __launch_bounds__(256) void kg_row_g(const GroupTask<RowParams>* __restrict__ tasks,
                                                const uint16_t* __restrict__ bt) {
  const GroupTask<RowParams>& T = group_task(tasks, bt);
  row_g_body<MODE, ST, STATS, RW>(T.p, T.gp, group_block(T));
}
__global__ __launch_bounds__(256) void kg_colg_fwd(const GroupTask<ColParams>* __restrict__ tasks,
                                                  const uint16_t* __restrict__ bt) {
  const GroupTask<ColParams>& T = group_task(tasks, bt);
  colg_fwd_body(T.p, T.gp, group_block(T));
}
__global__ __launch_bounds__(256) void kg_colg_syn(const GroupTask<ColParams>* __restrict__ tasks,
                                                  const uint16_t* __restrict__ bt) {
  const GroupTask<ColParams>& T = group_task(tasks, bt);
  colg_syn_body(T.p, T.gp, group_block(T));
}
__global__ __launch_bounds__(256) void kg_colg_ana(const GroupTask<ColParams>* __restrict__ tasks,
                                                  const uint16_t* __restrict__ bt) {
  const GroupTask<ColParams>& T = group_task(tasks, bt);
  colg_ana_body(T.p, T.gp, group_block(T));
}
__global__ __launch_bounds__(256) void kg_colg_final(const GroupTask<ColParams>* __restrict__ tasks,
                                                    const uint16_t* __restrict__ bt) {
  const GroupTask<ColParams>& T = group_task(tasks, bt);
  colg_final_body(T.p, T.gp, group_block(T));
}

// ---- pixel step (any size)
template <bool STATS, bool HAVE_Z>
__global__ __launch_bounds__(256) void kg_pixel(const GroupTask<PixParams>* __restrict__ tasks,
                                                const uint16_t* __restrict__ bt) {
  const GroupTask<PixParams>& T = group_task(tasks, bt);
  pixel_body<STATS, HAVE_Z>(T.p, group_block(T));
}

}  // namespace shs
