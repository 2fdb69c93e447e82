// Launcher of the grouped batch family (own translation unit).
#include "hdc_launch.hpp"

namespace hdc {

hdc_status run_batch(const hdc_functor* f, const hdc_functor& g, hdc_dtype dt, hdc_accum acc,
                     const hdc_batch_call* calls, const int32_t* grp, int ng, void* ws, size_t ws_bytes,
                     const Tuning& t, hipStream_t st) {
  if (dt == HDC_I32) {
    return with_int_fn(g, [&](auto gf) -> hdc_status {
      if (!f) return launch_batch<IntIdentity, decltype(gf), I32, IntAcc>(IntIdentity{}, gf, calls, grp, ng, ws, ws_bytes, t, st);
      return with_int_fn(*f, [&](auto mf) {
        return launch_batch<decltype(mf), decltype(gf), I32, IntAcc>(mf, gf, calls, grp, ng, ws, ws_bytes, t, st);
      });
    });
  }
  return with_float_storage(dt, [&](auto s) {
    using S = decltype(s);
    return with_float_fn(g, [&](auto gf) -> hdc_status {
      using G = decltype(gf);
      auto run = [&](auto a) -> hdc_status {
        using Acc = decltype(a);
        if constexpr (G::binary) {
          return fail(HDC_ERR_UNSUPPORTED, "PRODUCT is not a batch fold term");
        } else {
          if (!f) return launch_batch<Identity, G, S, Acc>(Identity{}, gf, calls, grp, ng, ws, ws_bytes, t, st);
          return with_float_fn(*f, [&](auto mf) -> hdc_status {
            using FM = decltype(mf);
            if constexpr (FM::binary)
              return fail(HDC_ERR_UNSUPPORTED, "PRODUCT cannot be mapped");
            else
              return launch_batch<FM, G, S, Acc>(mf, gf, calls, grp, ng, ws, ws_bytes, t, st);
          });
        }
      };
      if (acc == HDC_ACC_COMPENSATED) return run(CompAcc{});
      return run(PlainAcc{});
    });
  });
}

}  // namespace hdc
