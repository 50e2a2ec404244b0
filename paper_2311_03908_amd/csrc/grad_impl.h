// Kinetic-parameter gradient (adjoint) driver of Ctx<T>; included by capi.hip.
template <typename T>
int Ctx<T>::grad(const dem_grad_spec *s, const dem_gas *g, const double *theta, double *J, double *gr) {
  (void)s; (void)g; (void)theta; (void)J; (void)gr;
  return fail(DEMRX_EINVAL, "dem_grad unavailable");
}
