// Host helpers of the C ABI shared by its translation units (not public).
#pragma once

#include <string>
#include <vector>

#include "launch.h"
#include "status.h"

namespace bard {

// Record `msg` as the calling thread's last error and return `code`.
int fail(int code, const std::string& msg);
// BARD_E_DEVICE if an earlier asynchronous device error is pending (and clear it).
int check_device_state();
// Largest dynamic LDS allocation of one workgroup on device `dev`.
size_t lds_limit(int dev);
// True if `st` is being captured into a HIP graph (then nothing may be
// allocated or copied synchronously on its behalf).
bool capturing(hipStream_t st);
// Upload the model's tables to the current device (once per device).  On a
// first use while `st` is being captured: BARD_E_CAPTURE.
int ensure_device(bard_model* m, DeviceCopy** out, hipStream_t st);
// Device image of the Jacobian output lists for an end-effector set (cached
// per set); BARD_E_CAPTURE as for ensure_device.
int ensure_ee(bard_model* m, DeviceCopy* dc, int n_ee, const int32_t* ee_body, DevEE* out, hipStream_t st);
// Waves per workgroup for the phases after the level sweep (rs: scalar bytes).
int out_waves(int rs);

// Largest trees the specialiser takes: depth, and dofs times ancestor bodies
// summed over the tree (the mass-matrix walks of the generated code).
constexpr int kSpecMaxDepth = 32;
constexpr int kSpecMaxWalkSteps = 1500;
// Model-specialised chain kernels (specialize.cpp).  Key of one (precision,
// frame, end-effector set) in DeviceCopy::spec.
std::string spec_key(int dtype, int frame, const std::vector<int>& ee, int form);
// Batch tiers of the routing: [0, 4096), [4096, 16384), [16384, 65536),
// [65536, inf); autotuning times each at its lower bound (1024 for the first).
constexpr int kSpecTiers = 4;
constexpr int64_t kSpecTierBatch[kSpecTiers] = {1024, 4096, 16384, 65536};
int spec_tier(int64_t B);
// Forms of a specialised kernel: 0 split over waves by limbs, 1 one wave
// over the whole tree, 2 split and, per 64 instances, two workgroups (the
// torques in one, the mass matrix and Jacobians in the other), 3 split and
// three workgroups (torques, mass matrix, Jacobians).
constexpr int kSpecForms = 4;
// Source text of the kernel for one (end-effector set, frame, precision, form).
std::string spec_chain_source(const bard_model* m, const std::vector<int>& ee, int frame, bool fp64, int form);
// Source text of the specialised forward-dynamics (ABA) kernel of a tree.
// Single-operator specialised kernels (the chain kernel's code for one
// output: ops 1 torques, 2 mass matrix, 4 Jacobians of ee in frame; split
// over waves by limbs for form 0, one wave for form 1): source, key,
// compile-and-load, and the kernel a bard_rnea / bard_crba / bard_jacobian
// call routes to.
std::string spec_op_source(const bard_model* m, bool fp64, int form, int ops, const std::vector<int>& ee, int frame);
std::string spec_op_key(int ops, int dtype, int form, const std::vector<int>& ee, int frame);
int spec_prepare_op(bard_model* m, DeviceCopy* dc, int dtype, int form, int ops, const std::vector<int>& ee,
                    int frame, bool load, SpecKernel** out);
SpecKernel* spec_lookup_op(bard_model* m, DeviceCopy* dc, int dtype, int ops, const std::vector<int>& ee, int frame,
                           int64_t B);
std::string spec_aba_source(const bard_model* m, bool fp64, bool split);
// Multi-tree plan kernel (bard_spec_plan): every model's specialised chain
// code in one launch over [K][batch] arrays, each tree split over at most
// max_waves waves; *waves per workgroup and *blocks of the launch.
// spec_plan_build compiles and loads it on the current device (sk->mod,
// sk->fn; the caller unloads sk->mod).
std::string spec_plan_source(const std::vector<bard_model*>& ms, const std::vector<std::vector<int>>& ee,
                             const std::vector<int64_t>& batch, bool fp64, int max_waves, int* waves,
                             int64_t* blocks);
int spec_plan_build(const std::vector<bard_model*>& ms, const std::vector<std::vector<int>>& ee,
                    const std::vector<int64_t>& batch, bool fp64, int max_waves, SpecKernel* sk, int64_t* blocks);
// The per-model argument record of the multi-tree kernel (its PlanIO).
template <class Real>
struct SpecPlanIO {
  const Real* q;
  const Real* qd;
  const Real* qdd;
  Real* tau;
  Real* M;
  Real* J;
  Real g[4];
};

int spec_aba_waves(const bard_model* m, bool fp64, bool split);
// Waves per workgroup of that kernel (64 instances per workgroup).
int spec_waves(const bard_model* m, bool fp64, int form);
// Whether the tree has a plan for the form (the dual form needs a split plan).
bool spec_form_ok(const bard_model* m, bool fp64, int form);
// Number of structural-zero rows (M entries of unrelated dofs, J rows off an
// end effector's path) the kernel writes.
int spec_zero_rows(const bard_model* m, const std::vector<int>& ee);
// Compile source to a gfx950 code object with hipRTC (no device needed).
int spec_compile(const std::string& src, std::vector<char>* code, std::string* log);
// Compile (once) and, if `load`, load on the device of `dc`; *out points into dc->spec.
int spec_prepare(bard_model* m, DeviceCopy* dc, int dtype, int frame, const std::vector<int>& ee, int form,
                 bool load, SpecKernel** out);
// The routed specialised kernel for a chain call of batch B, or null.
SpecKernel* spec_lookup(bard_model* m, DeviceCopy* dc, int dtype, int frame, int n_ee, const int32_t* ee,
                        int64_t B);
// The specialised forward-dynamics kernel: compile/load, routed lookup for a
// batch, whether a call's lane offsets fit 32 bits, launch with bard_aba's
// arguments.
std::string spec_aba_key(int dtype);
int spec_prepare_aba(bard_model* m, DeviceCopy* dc, int dtype, bool load, SpecKernel** out);
SpecKernel* spec_lookup_aba(bard_model* m, DeviceCopy* dc, int dtype, int64_t B);
template <class Real>
bool spec_aba_fits(const Args<Real>& a);
template <class Real>
int spec_aba_launch(const SpecKernel* sk, const Args<Real>& a, const double g[3], hipStream_t st);
// Largest tree depth the specialised forward-dynamics kernel takes (the state
// of the bodies on the current path stays in registers).
constexpr int kSpecAbaMaxDepth = 16;
// Launch a specialised chain kernel with a chain call's arguments.
template <class Real>
int spec_launch(const SpecKernel* sk, const Args<Real>& a, const double g[3], hipStream_t st);
// Whether every lane's byte offset into each array of a chain call, and every
// output row's offset plus the lane's, fits the 32 bits the specialised
// kernels address with (else the generic kernel runs).
template <class Real>
bool spec_fits(const Args<Real>& a, int nv, int n_ee, int n_pose = 0);  // n_pose: bodies whose poses are written

}  // namespace bard
