// Collision and adjoint pipelines, float, padded grid P = 128: every compiled tile shape.
#include "qb_pipelines.hpp"

template bool collision_pipeline<float, 128, 32>(qb_plan_s*, const float*, float*, int, int, hipStream_t);
template bool collision_vjp_pipeline<float, 128, 32>(qb_plan_s*, const float*, const float*, float*, int, int,
                                                   hipStream_t);
template bool collision_pipeline<float, 128, 16>(qb_plan_s*, const float*, float*, int, int, hipStream_t);
template bool collision_vjp_pipeline<float, 128, 16>(qb_plan_s*, const float*, const float*, float*, int, int,
                                                   hipStream_t);
