// Learned proposal: affine-coupling flow on the 11 standardized parameters
// (host-side interface between the flow and the sampler translation units).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct pes_flow;

namespace pes {

// log q(theta) of the flow for n rows of theta [n][11] (FP64 in and out);
// z (may be null) receives the latent point.
int flow_forward(pes_flow* f, const double* theta, int64_t n, double* z, double* logq, hipStream_t s);
// theta = inverse map of z [n][11]; logdet (may be null) receives the log
// determinant of the normalizing map at theta (in the standardized space).
int flow_inverse(pes_flow* f, const double* z, int64_t n, double* theta, double* logdet, hipStream_t s);
// Makes the workspace hold n rows (allocates; not for use under capture).
int flow_reserve(pes_flow* f, int64_t n);
// Count of workspace reallocations: a captured graph that reads the workspace
// is valid only while this is unchanged.
uint64_t flow_generation(const pes_flow* f);

}  // namespace pes
