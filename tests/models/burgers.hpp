// Inviscid Burgers equation dq/dt + d(q^2/2)/dx = 0: a user model for the
// runtime-compiled step (not a model compiled into the library).
struct UserPDE {
  static constexpr int M = 1;
  static constexpr bool kSource = false, kNcp = false;
  static constexpr int kSrcVars = 0;
  template <class T> __device__ static void flux(const T* q, T* f, const PdeParams&) {
    f[0] = T(0.5) * q[0] * q[0];
  }
  template <class T> __device__ static T speed(const T* q, const PdeParams&) { return dabs(q[0]); }
  __device__ static bool admissible(const double* q, const PdeParams&) { return isfinite(q[0]); }
  __device__ static constexpr double diss(int) { return 1.0; }
};
