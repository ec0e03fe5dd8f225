// Closure network for a coarse periodic 2D field (see cnn.hip): host interface.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>

namespace sps {

class Cnn {
 public:
  // batch images of H x W (W a multiple of 32), 32 hidden channels
  Cnn(int batch, int H, int W, hipStream_t s);
  ~Cnn();
  static int nparam();
  // parameters: FP64 device vector (w1, b1, w2, b2, w3, b3) rounded into the stored tables
  void set_params(const double* theta_dev);
  // y = scale * net(x) (or y += ...), x and y FP64 device images [batch][H][W]
  void forward(const double* x, double* y, double scale, bool accumulate);
  // xb = xscale * (d net / d x)^T yb (or +=), th_bar += (d net / d theta)^T yb (th_bar nullable)
  void vjp(const double* x, const double* yb, double* xb, double xscale, bool accumulate, double* th_bar);
  // as vjp, with the parameter cotangent added to the network's own FP64 accumulators instead
  // (chunk partials, one owner per slot); grad_reset zeroes them, grad_flush adds their sum over
  // chunks (fixed order) to th_bar.  For sums over many calls, e.g. every step of a reverse sweep.
  void vjp_accumulate(const double* x, const double* yb, double* xb, double xscale, bool accumulate);
  void grad_reset();
  void grad_flush(double* th_bar);

 private:
  void backward(const double* x, const double* yb, double* xb, double xscale, bool accumulate, bool add);
  struct Impl;
  std::unique_ptr<Impl> p_;
};

}  // namespace sps
