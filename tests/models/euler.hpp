// The 1-D Euler gas (Sec. 2, eq. system_of_equations) written as a user model,
// in the same arithmetic as the compiled-in model, so the runtime-compiled
// step can be compared with the library's own.
struct UserPDE {
  static constexpr int M = 3;
  static constexpr bool kSource = false, kNcp = false;
  static constexpr int kSrcVars = 0;
  template <class T> __device__ static void flux(const T* q, T* f, const PdeParams& p) {
    const T u = q[1] * recip(q[0]);
    const T pr = T(p.gamma - 1.0) * (q[2] - T(0.5) * q[1] * u);
    f[0] = q[1];
    f[1] = q[1] * u + pr;
    f[2] = u * (q[2] + pr);
  }
  template <class T> __device__ static T speed(const T* q, const PdeParams& p) {
    const T ri = recip(q[0]);
    const T u = q[1] * ri;
    const T pr = T(p.gamma - 1.0) * (q[2] - T(0.5) * q[1] * u);
    return dabs(u) + sqrt(T(p.gamma) * pr * ri);
  }
  __device__ static bool admissible(const double* q, const PdeParams& p) {
    const double u = q[1] * recip(q[0]);
    const double pr = (p.gamma - 1.0) * (q[2] - 0.5 * q[1] * u);
    return isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2]) && q[0] > 0.0 && pr > 0.0;
  }
  __device__ static constexpr double diss(int) { return 1.0; }
};
