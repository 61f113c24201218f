// Launch sequences of the collision operator and of its transpose for one
// tile shape; included by the qb_tiles_*.hip units, which instantiate them.
#pragma once
#include "qb_plan.hpp"

// C[w] for the cells [cell0, cell0 + ncells) of the state arrays w, c
// (ncells <= wcells; the workspace holds the chunk's cells from index 0)
template <typename T, int P, int E>
bool collision_pipeline(qb_plan_s* pl, const T* w, T* c, int ncells, int cell0, hipStream_t s) {
  constexpr int NT = qb::Fft2<T, P, E>::NT;
  DevPlan<T> d = devplan<T>(pl, pl->cur_tab);
  int id = pl->begin(QB_K_DFT_IN, s);
  hipLaunchKernelGGL((qb::k_dft_in<T, P, E>), dim3(ncells), dim3(NT), 0, s, d, w, cell0);
  pl->end(id, s);
  // persistent launches: at most the workgroups that are resident at once
  // (rounded down to a multiple of 8), grid-striding over the task list
  auto grid = [&](int ntask, const void* kern) {
    return pl->persistent ? std::min(ntask, persistent_grid(kern, NT)) : ntask;
  };
  id = pl->begin(QB_K_TERMS, s);
  hipLaunchKernelGGL((qb::k_terms<T, P, E>), dim3(grid(ncells * qb::kTermPlanes, (const void*)qb::k_terms<T, P, E>)), dim3(NT),
                     0, s, d, ncells);
  pl->end(id, s);
  id = pl->begin(QB_K_I3, s);
  if (pl->i3_pair)
    hipLaunchKernelGGL((qb::k_i3<T, P, E, true>), dim3(grid(ncells * d.J, (const void*)qb::k_i3<T, P, E, true>)),
                       dim3(NT), 0, s, d, ncells);
  else
    hipLaunchKernelGGL((qb::k_i3<T, P, E, false>), dim3(grid(ncells * d.J, (const void*)qb::k_i3<T, P, E, false>)),
                       dim3(NT), 0, s, d, ncells);
  pl->end(id, s);
  const size_t nel = (size_t)ncells * P * P;
  hipLaunchKernelGGL((qb::k_assemble<T, P, E>), dim3(blocks(nel, 256)), dim3(256), 0, s, d, ncells);
  id = pl->begin(QB_K_COMBINE, s);
  hipLaunchKernelGGL((qb::k_combine<T, P, E>), dim3(ncells), dim3(NT), 0, s, d, c, cell0);
  pl->end(id, s);
  return hip_ok(hipGetLastError(), "collision launch");
}

// out = C'(w)^T lam for cells [0, ncells) (Pauli state layout, gradients)
template <typename T, int P, int E>
bool collision_vjp_pipeline(qb_plan_s* pl, const T* w, const T* lam, T* out, int ncells, int cell0,
                            hipStream_t s) {
  constexpr int NT = qb::Fft2<T, P, E>::NT;
  DevPlan<T> d = devplan<T>(pl, pl->vjp_tab);
  int id = pl->begin(QB_K_DFT_IN, s);
  hipLaunchKernelGGL((qb::k_dft_in<T, P, E>), dim3(ncells), dim3(NT), 0, s, d, w, cell0);
  pl->end(id, s);
  // the forward I_1 / I_4 / I_2 fields are formed inside k_terms_vjp
  id = pl->begin(QB_K_ADJOINT, s);
  hipLaunchKernelGGL((qb::k_lam_in<T, P, E>), dim3(ncells), dim3(NT), 0, s, d, lam, cell0);
  const size_t nel = (size_t)ncells * P * P;
  hipLaunchKernelGGL((qb::k_assemble_vjp<T>), dim3(blocks(nel, 256)), dim3(256), 0, s, d, ncells, P * P, 0);
  hipLaunchKernelGGL((qb::k_terms_vjp<T, P, E>), dim3(ncells * qb::kTermsVjpTasks), dim3(NT), 0, s, d);
  hipLaunchKernelGGL((qb::k_assemble_vjp<T>), dim3(blocks(nel, 256)), dim3(256), 0, s, d, ncells, P * P, 1);
  pl->end(id, s);
  id = pl->begin(QB_K_I3_ADJOINT, s);
  if (pl->vjp_variant == 1)
    hipLaunchKernelGGL((qb::k_i3_vjp_reg<T, P, E, true>), dim3(ncells * d.J), dim3(NT), 0, s, d, ncells);
  else
    hipLaunchKernelGGL((qb::k_i3_vjp_reg<T, P, E, false>), dim3(ncells * d.J), dim3(NT), 0, s, d, ncells);
  pl->end(id, s);
  id = pl->begin(QB_K_ADJOINT, s);
  hipLaunchKernelGGL((qb::k_grad_pre<T>), dim3(blocks(nel * 8, 256)), dim3(256), 0, s, d, ncells, P * P);
  hipLaunchKernelGGL((qb::k_grad_out<T, P, E>), dim3(ncells), dim3(NT), 0, s, d, out, cell0);
  pl->end(id, s);
  return hip_ok(hipGetLastError(), "collision adjoint launch");
}

